"""FP32 rays test the horizon as u >= uh32, where uh32 is the smallest float at
or above uh = 1/(2M) (the host rounds 1/(2M) to float and steps up one ulp if
the rounding went down).  For every float u this decides exactly as the FP64
test (double)u >= uh.  Checked here for many M at the floats around uh."""
import numpy as np


def uh32_of(uh: float) -> np.float32:
    f = np.float32(uh)
    if float(f) < uh:
        f = np.nextafter(f, np.float32(np.inf))
    return f


def test_float_horizon_test_decides_as_fp64():
    rng = np.random.default_rng(7)
    masses = np.concatenate([[1.0, 0.5, 2.0, 3.0, 1e-3, 1e3, 0.1, 7.0],
                             rng.uniform(0.01, 100.0, 2000)])
    for M in masses:
        uh = 1.0 / (2.0 * M)
        t = uh32_of(uh)
        u = t
        for _ in range(4):  # a few floats below the threshold
            u = np.nextafter(u, np.float32(-np.inf))
        for _ in range(9):  # ... through a few above it
            assert (u >= t) == (float(u) >= uh), (M, float(u))
            u = np.nextafter(u, np.float32(np.inf))


def test_rounding_to_nearest_alone_would_not_do():
    # with plain rounding, some M put the float threshold below uh, and a
    # float u equal to it would count as captured though (double)u < uh
    bad = 0
    for M in np.random.default_rng(3).uniform(0.01, 100.0, 2000):
        uh = 1.0 / (2.0 * M)
        f = np.float32(uh)
        if float(f) < uh and (f >= f) != (float(f) >= uh):
            bad += 1
    assert bad > 0
