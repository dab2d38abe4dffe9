"""The kernels take a pixel's row as trunc(fma(i, 1/W, 1/(2W))), one FP64 fma
with the rounded reciprocal, instead of an integer division.  The argument
that this is exact for every index i < 2^31 and every width W: the fma's one
rounding and the reciprocal's leave the quotient within 2^-52 relative, hence
within 2^-21 / W, while (i + 1/2) / W lies at least 1/(2W) from every integer.
These tests redo the fma with exact rationals rounded once to double (what
the hardware fma does) at the boundary indices of many widths."""
from fractions import Fraction



def fma_then_round(a: float, b: float, c: float) -> float:
    return float(Fraction(a) * Fraction(b) + Fraction(c))  # exact, then rounded to nearest


def row_of(i: int, W: int) -> int:
    inv = 1.0 / W
    return int(fma_then_round(float(i), inv, 0.5 * inv))  # int() truncates


def boundary_indices(W: int):
    top = 2**31 - 1
    last_row = top // W
    for k in (0, 1, 2, 3, last_row - 1, last_row):
        for off in (-1, 0, 1, W - 2, W - 1):
            i = k * W + off
            if 0 <= i <= top:
                yield i
    yield top


WIDTHS = sorted(set(list(range(1, 400)) + [3840, 4096, 7680, 2**16 - 1, 2**16, 2**16 + 1,
                                            10**6 + 3, 2**20 + 1, 2**24 - 3, 2**30 + 7,
                                            2**31 - 1]))


def test_row_from_one_fma_is_exact():
    for W in WIDTHS:
        for i in boundary_indices(W):
            assert row_of(i, W) == i // W, (i, W)


def test_truncating_a_plain_product_would_not_be():
    # without the half-step offset, a row boundary i = k W can land below k
    bad = [(k * W, W) for W in WIDTHS[:399] for k in range(1, 200)
           if int(fma_then_round(float(k * W), 1.0 / W, 0.0)) != k]
    assert bad, "expected some widths where i * (1/W) rounds below the row boundary"


def test_row_is_exact_for_a_4k_frame_sampled_densely():
    W = 3840
    for i in range(0, 3840 * 2160, 997):
        for j in (i, i + W - 1 - (i % W)):
            assert row_of(j, W) == j // W
