"""Independent closed forms and quadratures of the photon orbit, used to pin the
oracle.  Nothing here calls the oracle or the GPU library.

The orbit equation u'' + u = 3 M u^2 has the first integral
    (du/dphi)^2 = P(u) = 1/b^2 - u^2 + 2 M u^3,
so the azimuth swept between two radii is an integral of du / sqrt(P(u)).
Near a turning point u2 (a simple root of P) the substitution u = u2 - s^2
removes the inverse-square-root singularity:
    P(u2 - s^2) = 2 M s^2 (u2 - u1 - s^2) (u3 - u2 + s^2),
where u1 < 0 < u2 < u3 are the three real roots (for b > 3 sqrt(3) M).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

B_CRIT = 3.0 * math.sqrt(3.0)


def roots(M: float, b: float):
    """Real roots u1 < u2 < u3 of 2 M u^3 - u^2 + 1/b^2 (M > 0, b > b_c M)."""
    r = np.roots([2.0 * M, -1.0, 0.0, 1.0 / b**2])
    r = np.sort(r.real)
    out = []
    for x in r:  # Newton polish in float64
        for _ in range(4):
            p = 2 * M * x**3 - x**2 + 1.0 / b**2
            dp = 6 * M * x**2 - 2 * x
            if dp != 0:
                x = x - p / dp
        out.append(x)
    return out


def psi(M: float, b: float, u_lo: float) -> float:
    """Azimuth swept between u_lo and the turning point u2 (u_lo <= u2)."""
    if M == 0.0:
        u2 = 1.0 / b
        f = lambda s: 2.0 / math.sqrt(2.0 * u2 - s * s)
    else:
        u1, u2, u3 = roots(M, b)
        f = lambda s: 2.0 / math.sqrt(2.0 * M * (u2 - u1 - s * s) * (u3 - u2 + s * s))
    smax = math.sqrt(max(u2 - u_lo, 0.0))
    val, _ = integrate.quad(f, 0.0, smax, epsabs=1e-15, epsrel=1e-14, limit=400)
    return val


def turning_point(M: float, b: float) -> float:
    return 1.0 / b if M == 0.0 else roots(M, b)[1]


def exit_phi(M: float, b: float, r0: float, r_sky: float, ingoing: bool) -> float:
    """Azimuth at which the ray reaches the sky sphere (b > critical when
    ingoing; any b for outgoing rays)."""
    u0, us = 1.0 / r0, 1.0 / r_sky
    if ingoing:
        return psi(M, b, u0) + psi(M, b, us)
    P = lambda u: 1.0 / b**2 - u * u + 2.0 * M * u**3
    val, _ = integrate.quad(lambda u: 1.0 / math.sqrt(P(u)), us, u0, epsabs=1e-15,
                            epsrel=1e-14, limit=400)
    return val


def phi_at_u(M: float, b: float, r0: float, u: float, after_turn: bool) -> float:
    """Azimuth at which an ingoing ray from r0 reaches u, before or after the
    turning point."""
    u0 = 1.0 / r0
    if after_turn:
        return psi(M, b, u0) + psi(M, b, u)
    return psi(M, b, u0) - psi(M, b, u)


def weak_field_sweep(M: float, b: float, r0: float, r_sky: float) -> float:
    """First-order solution u = sin(phi)/b + (M/b^2)(1 + cos^2 phi), symmetric
    about the periapsis: sweep = pi - a(r_sky) - a(r0) with
    a(r) = asin(b/r - (M/b)(2 - b^2/r^2)).  Error is O((M/b)^2)."""
    a = lambda r: math.asin(b / r - (M / b) * (2.0 - b * b / (r * r)))
    return math.pi - a(r_sky) - a(r0)


def shadow_sin2(M: float, r0: float) -> float:
    """sin^2 of the shadow half-angle seen from r0 under the straight-line
    initial direction: the ray is captured iff sin^2(alpha) below this, where
    alpha is the angle to the inward radial (from 1/b^2 = u0^2/sin^2 - 2 M u0^3
    and b_c^2 = 27 M^2)."""
    u0 = 1.0 / r0
    return u0 * u0 / (1.0 / (27.0 * M * M) + 2.0 * M * u0**3)
