"""Why the FP32 integrator's horizon test cannot change a ray's class.

FP32 rays are the rays outside the critical band, |b - 3 sqrt(3) M| >= 0.05 M,
with b computed in FP64 at set-up.  Their horizon test is v >= 3/2 in FP32
(v = 3 M u; u = 1/(2M) is v = 3/2).  From Eq. (1)'s first integral,
w^2 = 1/b^2 - u^2 + 2 M u^3 along a ray:
  - above the band the orbit turns at u2, the smallest positive root of
    2 M u^3 - u^2 + 1/b^2, and u2 < 1/(3M): v never exceeds 3 M u2 < 1, a
    margin of more than 0.5 below the threshold, which an integrator that
    keeps v to about 1e-6 relative cannot cross;
  - below the band an ingoing ray has no turning point before the horizon
    (1/b^2 - u^2 + 2 M u^3 > 0 for every u up to 1/(2M)), so v reaches 3/2 at
    some step and FP32 only decides at which step the capture is recorded.
These are checked here from the cubic itself (numpy's polynomial roots), not
from the oracle or the kernels.  The GPU parity tests check the classes
themselves, bit for bit outside the band.
"""
import math

import numpy as np

M = 1.0
BC = 3.0 * math.sqrt(3.0) * M
BAND = 0.05 * M


def periapsis_v(b):
    """3 M u2 with u2 the smallest positive real root of 2 M u^3 - u^2 + 1/b^2
    (nan if there is none: no turning point)."""
    r = np.roots([2.0 * M, -1.0, 0.0, 1.0 / (b * b)])
    pos = sorted(x.real for x in r if abs(x.imag) < 1e-12 and x.real > 0)
    return 3.0 * M * pos[0] if pos else math.nan


def test_turning_point_stays_far_below_the_horizon_above_the_band():
    bs = np.concatenate([BC + BAND + np.geomspace(1e-9, 1.0, 200), np.geomspace(BC + 1.1, 1e3, 200)])
    v2 = np.array([periapsis_v(b) for b in bs])
    assert np.all(np.isfinite(v2))
    assert v2.max() < 1.0            # inside the photon sphere never reached
    assert 1.5 - v2.max() > 0.5      # margin to the FP32 threshold v = 3/2
    # closed form at the band edge: close to the photon sphere, v2 near 1
    assert 0.8 < periapsis_v(BC + BAND) < 1.0
    # and v2 -> 1 (r_min -> 3M) as b -> b_c from above
    assert abs(periapsis_v(BC * (1 + 1e-9)) - 1.0) < 1e-3


def test_no_turning_point_before_the_horizon_below_the_band():
    u = np.linspace(0.0, 1.0 / (2.0 * M), 20001)
    for b in np.concatenate([np.linspace(1e-3, BC - BAND, 300), [BC - BAND]]):
        w2 = 1.0 / (b * b) - u * u + 2.0 * M * u ** 3
        assert w2.min() > 0.0, b
        assert math.isnan(periapsis_v(b)) or periapsis_v(b) > 1.5


def test_margin_detects_a_wrong_threshold():
    """Negative control: with the horizon threshold taken at the photon
    sphere (v = 1) instead of v = 3/2, band-edge rays would come within 0.12
    of it, so the margin claimed above is not vacuous."""
    assert 1.0 - periapsis_v(BC + BAND) < 0.12
