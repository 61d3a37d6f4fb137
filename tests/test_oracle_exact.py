"""Pins of the exact-product yardstick (oracle/exact.py) used for the slice path."""

from fractions import Fraction

from mpmath import mp, mpf, fsum

from oracle import exact, mpnum
from paper_1410_1599_amd import inputs as I


def test_exact_dot_matches_rational_sum_and_mpmath():
    p = 256
    A = I.log_uniform(3, 50, p, 1)
    B = I.log_uniform(50, 3, p, 2)
    Ao, Bo = I.from_planes(A, p), I.from_planes(B, p)
    mp.prec = 4000
    for i in range(3):
        for j in range(3):
            n, f = exact.exact_dot(Ao[i], [Bo[k][j] for k in range(50)], p)
            fr = sum((mpnum.to_fraction(Ao[i][k], p) * mpnum.to_fraction(Bo[k][j], p) for k in range(50)), Fraction(0))
            assert Fraction(n) * Fraction(2) ** f == fr
            # mpmath's fsum at a precision far above the spread is exact here
            s = fsum(mpf(Ao[i][k][0]) * mpf(2) ** (Ao[i][k][1] - p) * mpf(Bo[k][j][0]) * mpf(2) ** (Bo[k][j][1] - p) for k in range(50))
            assert s == mpf(n) * mpf(2) ** f
            c = exact.exact_entry(Ao, Bo, i, j, p)
            assert exact.ulp_error(c, n, f, p) <= Fraction(1, 2)


def test_ulp_error_of_neighbours():
    p = 128
    x = (3 << (p - 2), 0)               # 0.75
    n, f = x[0], x[1] - p
    assert exact.ulp_error(x, n, f, p) == 0
    up = (x[0] + 1, 0)
    assert exact.ulp_error(up, n, f, p) == 1
    assert exact.ulp_error(mpnum.ZERO, 0, 0, p) == 0


def test_slice_model_equals_exact_rounding_when_window_covers_spread():
    p = 128
    A = I.from_planes(I.log_uniform(4, 30, p, 3, -6, 6), p)
    B = I.from_planes(I.log_uniform(30, 5, p, 4, -6, 6), p)
    WA, WB = exact.window_widths(A, B, p, 64)
    assert WA <= p + 12 and WB <= p + 12
    for i in range(4):
        for j in range(5):
            assert exact.slice_model_entry(A, B, i, j, p, WA, WB) == exact.exact_entry(A, B, i, j, p)


def test_slice_model_truncates_toward_zero_below_the_window():
    # p = 32 (model only): row max 2^0; with W = p + 2 an entry 2^-40 below
    # keeps nothing, one 3 binades below keeps its top 31 bits, truncated
    p = 32
    big = (1 << 31, 1)                    # 1.0
    tiny = ((1 << 31) | 1, -40)           # about 2^-41
    mid = (-((1 << 31) | 5), -2)          # about -2^-3, low bits set
    one = (1 << 31, 1)
    A = [[big, tiny, mid]]
    B = [[one], [one], [one]]
    got = exact.slice_model_entry(A, B, 0, 0, p, p + 2, p)
    # alpha = trunc(a * 2^(W - 1)) = trunc(a * 2^33)
    alpha = [(1 << 33), 0, -(((1 << 31) | 5) >> 1)]   # shift W - p - 3 = -1
    z = sum(alpha) * (1 << 31)            # beta = 2^31 for 1.0 with W_B = p, f = 1
    assert got == mpnum.rn(z, 1 + 1 - (p + 2) - p, p)
    assert exact.window_widths(A, B, p, 2) == (p + 2, p)
