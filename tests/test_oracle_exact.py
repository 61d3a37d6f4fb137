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
