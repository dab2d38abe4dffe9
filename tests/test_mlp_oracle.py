"""Pins of the FP64 surrogate-network oracle: finite differences, the Adam
closed form of a first step, loss special cases, feature/target identities,
bf16 rounding against torch, and the weak-field baseline against quadrature."""
import math

import numpy as np
import pytest

import quadrature as Q
from oracle import mlp_ref as R


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    b = np.where(rng.uniform(size=n) < 0.8, np.exp(rng.uniform(np.log(5.3), np.log(1000), n)),
                 rng.uniform(0.0, 5.1, n))
    r0 = rng.uniform(10, 200, n)
    esc = (b > R.B_CRIT).astype(float)
    t = rng.normal(size=n)
    return R.features(b, r0), t, esc, 1.0 - esc


def _loss(params, x, t, e, c):
    y, _ = R.forward(params, x)
    return R.loss_and_dy(y, t, e, c)[0]


def test_backward_matches_central_differences():
    """Analytic gradients of the loss against central differences in FP64
    (step 1e-6) on 40 random parameter entries across all eight tensors."""
    params = [p.astype(np.float64) for p in R.init_params(1)]
    params[7] += 0.3  # nonzero output bias
    for k in (1, 3, 5):
        params[k] += np.random.default_rng(k).normal(scale=0.1, size=params[k].shape)
    x, t, e, c = _batch(64, 2)
    y, cache = R.forward(params, x)
    # keep clear of ReLU kinks so the finite differences are smooth
    for z in (cache[1], cache[3], cache[5]):
        assert np.abs(z).min() > 1e-5
    _, dy = R.loss_and_dy(y, t, e, c)
    g = R.backward(params, cache, dy)
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(40):
        k = int(rng.integers(0, 8))
        idx = tuple(int(rng.integers(0, s)) for s in params[k].shape)
        pp = [p.copy() for p in params]
        pm = [p.copy() for p in params]
        pp[k][idx] += h
        pm[k][idx] -= h
        fd = (_loss(pp, x, t, e, c) - _loss(pm, x, t, e, c)) / (2 * h)
        assert abs(fd - g[k][idx]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, idx, fd, g[k][idx])


def test_adam_first_step_closed_form():
    """From m = v = 0 the first Adam step is lr * g / (|g| + eps): a step of
    (almost exactly) lr against the sign of each gradient entry."""
    p = [np.array([1.0, -2.0, 0.5])]
    g = [np.array([0.3, -4.0, 1e-3])]
    out, m, v = R.adam_step(p, g, [np.zeros(3)], [np.zeros(3)], step=1, lr=0.01)
    np.testing.assert_allclose(out[0], p[0] - 0.01 * g[0] / (np.abs(g[0]) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(out[0], p[0] - 0.01 * np.sign(g[0]), rtol=1e-6)
    np.testing.assert_allclose(m[0], 0.1 * g[0])
    np.testing.assert_allclose(v[0], 0.001 * g[0] ** 2)


def test_loss_special_cases():
    """Zero logit costs log 2 per sample whatever the label; an escaping
    sample predicted exactly costs nothing in the squared term; captured
    samples contribute no squared term."""
    y = np.array([[0.5, 0.0], [2.0, 0.0]])
    L, dy = R.loss_and_dy(y, [0.5, 99.0], [1.0, 0.0], [0.0, 1.0])
    assert abs(L - R.BCE_WEIGHT * math.log(2.0)) < 1e-15
    assert dy[0, 0] == 0.0 and dy[1, 0] == 0.0
    np.testing.assert_allclose(dy[:, 1], R.BCE_WEIGHT * np.array([0.5, -0.5]) / 2)


def test_forward_hand_network():
    """A network wired by hand: y0 = relu(relu(relu(f1))) , y1 = -f2 path."""
    W1 = np.zeros((2, 128)); W1[0, 0] = 1.0; W1[1, 1] = -1.0
    Wm = np.zeros((128, 128)); Wm[0, 0] = 1.0; Wm[1, 1] = 1.0
    W4 = np.zeros((128, 2)); W4[0, 0] = 2.0; W4[1, 1] = 1.0
    params = [W1, np.zeros(128), Wm, np.zeros(128), Wm, np.zeros(128), W4, np.array([0.25, -1.0])]
    y, _ = R.forward(params, np.array([[0.7, -0.3], [-0.2, 0.4]]))
    np.testing.assert_allclose(y, [[1.65, -0.7], [0.25, -1.0]])


def test_features_and_target_roundtrip():
    f = R.features([R.B_CRIT, R.B_CRIT + 0.05, 100.0], [10.0, 105.0, 200.0])
    assert f[0, 0] == 0.0 and abs(f[1, 0] - math.log(2.0) / 5) < 1e-15
    np.testing.assert_allclose(f[:, 1], [-1.0, 0.0, 1.0])
    b, r0 = np.array([6.0, 20.0, 300.0]), np.array([30.0, 150.0, 190.0])
    phi = np.array([4.0, 3.3, 3.2])
    np.testing.assert_allclose(R.predict_exit(b, r0, R.targets(b, r0, phi)), phi, rtol=1e-14)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.concatenate([np.random.default_rng(5).normal(size=1000).astype(np.float32),
                        np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -0.0, 65504.0], np.float32)])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(R.bf16_round(x), want)


def test_first_order_sweep_is_weak_field_accurate():
    """The baseline sweep1 agrees with the exact sweep (quadrature of the
    first integral) to O((M/b)^2): within 3 (15 pi / 4) / b^2."""
    for b in (40.0, 80.0, 150.0, 300.0):
        r0 = 180.0 if b < 180 else 400.0
        exact = Q.exit_phi(1.0, b, r0, R.R_SKY, True)
        assert abs(R.sweep_first_order(b, r0) - exact) < 3 * (15 * math.pi / 4) / b**2


def _dyadic_network(rng):
    """A network whose every activation and back-propagated gradient is exact
    in bf16: each unit reads exactly one unit of the layer below, through a
    power-of-two weight, with zero biases (scaled permutations), so values
    stay signed powers of two times the dyadic inputs."""
    params = []
    for k, (fi, fo) in enumerate(R.SHAPES):
        W = np.zeros((fi, fo), np.float32)
        src = rng.permutation(fo) % fi if fi < fo else rng.permutation(fi)[:fo]
        for j in range(fo):
            W[src[j], j] = rng.choice([-1.0, 1.0]) * 2.0 ** int(rng.integers(-2, 3))
        params += [W, np.zeros(fo, np.float32)]
    return params


def test_quantized_network_is_exact_where_nothing_rounds():
    """quantize=True only rounds: on a network and batch whose activations
    and gradients are all exact bf16 values it gives the same forward and
    backward bit for bit as the plain FP64 network."""
    rng = np.random.default_rng(3)
    p = _dyadic_network(rng)
    x = rng.choice([-1.0, -0.5, 0.25, 0.75, 1.5], size=(64, 2))
    dy = rng.choice([-2.0, -0.125, 0.0, 0.5, 1.0], size=(64, 2))
    y0, c0 = R.forward(p, x)
    y1, c1 = R.forward(p, x, quantize=True)
    np.testing.assert_array_equal(y0, y1)
    g0 = R.backward(p, c0, dy)
    g1 = R.backward(p, c1, dy, quantize=True)
    for a, b in zip(g0, g1):
        np.testing.assert_array_equal(a, b)
    assert any(np.abs(a).max() > 0 for a in g0)


def test_quantized_network_rounds_at_bf16_precision():
    """On a random network the rounded activations move the outputs by about
    bf16 precision (2^-9 relative per stored value).  Gradients move more: a
    ReLU whose input lies within rounding of zero can switch, and a switched
    unit changes its sample's whole contribution.  Away from such samples
    (every pre-activation at least 1e-2 of its layer's RMS from zero) the
    gradients too differ by about bf16 precision."""
    rng = np.random.default_rng(4)
    p = [R.bf16_round(a) for a in R.init_params(5)]
    for k in (1, 3, 5, 7):
        p[k] = R.bf16_round(rng.normal(scale=0.1, size=p[k].shape).astype(np.float32))
    x = rng.normal(size=(2048, 2))
    dy = rng.normal(size=(2048, 2)) / 256
    y0, c0 = R.forward(p, x)
    y1, c1 = R.forward(p, x, quantize=True)
    rel = np.abs(y1 - y0).max() / np.abs(y0).max()
    assert 1e-5 < rel < 2e-2, rel
    for a, b in zip(R.backward(p, c0, dy), R.backward(p, c1, dy, quantize=True)):
        rel = np.linalg.norm(a - b) / np.linalg.norm(a)
        assert 1e-5 < rel < 0.2, rel
    clear = np.ones(x.shape[0], bool)
    for z in (c0[1], c0[3], c0[5]):
        clear &= np.all(np.abs(z) >= 1e-2 * np.sqrt(np.mean(z * z)), axis=1)
    assert clear.sum() > 50
    y0, c0 = R.forward(p, x[clear])
    y1, c1 = R.forward(p, x[clear], quantize=True)
    for a, b in zip(R.backward(p, c0, dy[clear]), R.backward(p, c1, dy[clear], quantize=True)):
        rel = np.abs(a - b).max() / np.abs(a).max()
        assert rel < 2e-2, rel
