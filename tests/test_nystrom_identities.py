"""The identities behind the integrator's Nystrom form of the Dormand-Prince
5(4) step (the u component's derivative is w itself), checked with exact
rationals from the published tableau (Dormand & Prince 1980; Hairer, Norsett &
Wanner, Solving ODEs I, Sec. II.5), and the two forms compared on random
states of Eq. (1) in float64."""
from fractions import Fraction as F

import numpy as np

A = {(2, 1): F(1, 5), (3, 1): F(3, 40), (3, 2): F(9, 40), (4, 1): F(44, 45), (4, 2): F(-56, 15),
     (4, 3): F(32, 9), (5, 1): F(19372, 6561), (5, 2): F(-25360, 2187), (5, 3): F(64448, 6561),
     (5, 4): F(-212, 729), (6, 1): F(9017, 3168), (6, 2): F(-355, 33), (6, 3): F(46732, 5247),
     (6, 4): F(49, 176), (6, 5): F(-5103, 18656)}
B = {1: F(35, 384), 2: F(0), 3: F(500, 1113), 4: F(125, 192), 5: F(-2187, 6784), 6: F(11, 84)}
E = {1: F(71, 57600), 2: F(0), 3: F(-71, 16695), 4: F(71, 1920), 5: F(-17253, 339200),
     6: F(22, 525), 7: F(-1, 40)}


def a(k, m):
    """Row 7 of the extended tableau is b (first same as last)."""
    if k == 7:
        return B.get(m, F(0))
    return A.get((k, m), F(0))


def derived():
    c = {k: sum(a(k, j) for j in range(1, k)) for k in range(2, 8)}
    abar = {(k, m): sum(a(k, j) * a(j, m) for j in range(1, k)) for k in range(2, 7) for m in range(1, k)}
    bbar = {m: sum(B[j] * a(j, m) for j in range(1, 7)) for m in range(1, 7)}
    ebar = {m: sum(E[j] * a(j, m) for j in range(1, 8)) for m in range(1, 8)}
    return c, abar, bbar, ebar


def test_weights_sum_and_vanishing_terms():
    c, abar, bbar, ebar = derived()
    assert sum(B.values()) == 1 and sum(E.values()) == 0
    assert c[6] == 1 and c[7] == 1 and c[2] == F(1, 5) and c[5] == F(8, 9)
    # stage k uses g_1 .. g_(k-2) only; the solution g_1 .. g_5; the error g_1 .. g_6
    assert all(abar[(k, m)] == 0 for k in range(2, 7) for m in range(k - 1, k))
    assert bbar[6] == 0 and ebar[7] == 0
    assert bbar[2] == 0 and ebar[2] == 0
    assert abar[(3, 1)] == F(9, 200) and bbar[1] == B[1]


def test_forms_agree_on_random_states():
    c, abar, bbar, ebar = derived()
    fa = {k: float(v) for k, v in A.items()}
    rng = np.random.default_rng(7)
    n = 4000
    M3 = 3.0 * rng.uniform(0.0, 2.0, n)
    u = rng.uniform(1e-3, 0.3, n)
    w = rng.uniform(-0.3, 0.3, n)
    h = rng.uniform(1e-3, 1.0, n)
    g = lambda x: x * (M3 * x - 1.0)  # noqa: E731
    # standard form: u and w values of every stage
    us, ws, gs = {1: u}, {1: w}, {1: g(u)}
    for k in range(2, 7):
        us[k] = u + h * sum(fa.get((k, j), 0.0) * ws[j] for j in range(1, k))
        ws[k] = w + h * sum(fa.get((k, j), 0.0) * gs[j] for j in range(1, k))
        gs[k] = g(us[k])
    un = u + h * sum(float(B[j]) * ws[j] for j in range(1, 7))
    wn = w + h * sum(float(B[j]) * gs[j] for j in range(1, 7))
    ws[7], gs[7] = wn, g(un)
    eu = h * sum(float(E[j]) * ws[j] for j in range(1, 8))
    # Nystrom form: stage u values from g alone
    hw, h2 = h * w, h * h
    ns = {1: gs[1]}
    for k in range(2, 7):
        uk = u + float(c[k]) * hw + h2 * sum(float(abar[(k, m)]) * ns[m] for m in range(1, k))
        np.testing.assert_allclose(uk, us[k], rtol=1e-13, atol=1e-14)
        ns[k] = g(uk)
    un2 = u + hw + h2 * sum(float(bbar[m]) * ns[m] for m in range(1, 6))
    np.testing.assert_allclose(un2, un, rtol=1e-13, atol=1e-14)
    eu2 = h2 * sum(float(ebar[m]) * ns[m] for m in range(1, 7))
    # the error estimate is a difference of nearly equal sums: compare on the
    # scale of its terms
    scale = h * sum(abs(float(E[j])) * np.abs(ws[j]) for j in range(1, 8))
    assert np.max(np.abs(eu2 - eu) / scale) < 1e-13


def kernel_constants():
    """The constexpr coefficients of dp45 in the kernel source, evaluated."""
    import os
    import re
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = open(os.path.join(root, "paper_2507_16165_amd", "csrc", "bh_kernels.hip")).read()
    body = src[src.index("void dp45("):]
    body = body[:body.index("const T hw")]
    env = {}
    for stmt in re.findall(r"constexpr double ([^;]+);", body):
        for part in stmt.split(","):
            name, expr = (x.strip() for x in part.split("=", 1))
            assert re.fullmatch(r"[0-9a-zA-Z_.+\-*/ ()]+", expr), expr
            env[name] = eval(expr, {"__builtins__": {}}, dict(env))  # noqa: S307
    return env


def test_kernel_coefficients_are_the_derived_ones():
    """The tableau typed into the kernel, and the Nystrom coefficients it
    derives from it, equal the exact values (to double rounding)."""
    k = kernel_constants()
    c, abar, bbar, ebar = derived()
    want = {f"a{i}{j}": v for (i, j), v in A.items()}
    want.update({f"b{j}": v for j, v in B.items() if v != 0})
    want.update({f"e{j}": v for j, v in E.items() if v != 0})
    want.update({"c3": c[3], "c4": c[4], "c5": c[5]})
    want.update({f"A{i}{m}": abar[(i, m)] for i in range(3, 7) for m in range(1, i - 1)})
    want.update({"B1": bbar[1], "B3": bbar[3], "B4": bbar[4], "B5": bbar[5]})
    want.update({"E1": ebar[1], "E3": ebar[3], "E4": ebar[4], "E5": ebar[5], "E6": ebar[6]})
    assert set(want) == set(k), sorted(set(want) ^ set(k))
    for name, v in want.items():
        assert abs(k[name] - float(v)) <= 4e-16 * max(1.0, abs(float(v))), (name, k[name], float(v))
