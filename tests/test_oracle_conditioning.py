"""Exact condition numbers of the paper's Lotkin matrix (Section 4).

The closed form of the Hilbert inverse and the Sherman-Morrison step are
pinned against Gauss-Jordan inverses in exact rational arithmetic on small
n; then the n = 1024 values are compared with the figure the paper prints.
The paper gives 4.3 x 10^1576 for ||A||_1 ||A^-1||_1; exactly,
||A||_inf ||A^-1||_inf = 4.3 x 10^1567 (the printed mantissa, the exponent's
last two digits transposed) and ||A||_1 ||A^-1||_1 = 3.1 x 10^1565.  The
reading taken: the printed number is the infinity-norm condition number with
a transposed exponent; either way 8192 bits (2466 digits) leave about
2466 - 1566 = 900 correct digits for x, which the 8192-bit Lotkin LU on the
GPU reproduces (about 902 digits at n = 1024, column-wise)."""

from fractions import Fraction

import numpy as np
import pytest

from oracle import conditioning as C


@pytest.mark.parametrize("n", [1, 2, 3, 6, 9])
def test_hilbert_inverse_closed_form(n):
    H = [[Fraction(1, i + j - 1) for j in range(1, n + 1)] for i in range(1, n + 1)]
    inv = C.inverse_fraction(H)
    for j in range(1, n + 1):
        col = C._hilbert_inverse_column(n, j)
        for i in range(1, n + 1):
            assert inv[i - 1][j - 1] == C.hilbert_inverse_entry(n, i, j) == col[i - 1]


@pytest.mark.parametrize("n", [2, 3, 5, 8, 12])
def test_lotkin_conditions_match_gauss_jordan(n):
    A = C.lotkin(n)
    k1, kinf = C.lotkin_conditions(n)
    assert k1 == C.cond1(A)
    assert kinf == C.cond_inf(A)


def test_hilbert_inverse_recurrence_at_larger_n():
    n = 150
    for j in (1, 2, 75, 149, 150):
        col = C._hilbert_inverse_column(n, j)
        assert all(col[i - 1] == C.hilbert_inverse_entry(n, i, j) for i in (1, 2, 50, 149, 150))


def test_decimal_mantissa_exponent():
    assert C.decimal_mantissa_exponent(Fraction(43, 10) * Fraction(10) ** 1567) == (4.3, 1567)
    assert C.decimal_mantissa_exponent(Fraction(4349, 1000) * Fraction(10) ** 5) == (4.3, 5)
    assert C.decimal_mantissa_exponent(Fraction(9996, 1000)) == (1.0, 1)
    assert C.decimal_mantissa_exponent(Fraction(1, 400)) == (2.5, -3)


@pytest.mark.slow
def test_lotkin_1024_condition_numbers_against_the_paper():
    k1, kinf = C.lotkin_conditions(1024)
    assert C.decimal_mantissa_exponent(kinf) == (4.3, 1567)      # the paper: 4.3 x 10^1576
    assert C.decimal_mantissa_exponent(k1) == (3.1, 1565)


def test_random_matrix_condition_is_of_the_papers_order():
    """The paper's random matrix (n = 1024, entries in [-1, 1], seed unknown)
    has ||A||_1 ||A^-1||_1 = 4.4 x 10^6; a seeded uniform matrix of the same
    size lands within two decimal orders (float64 is ample at this size)."""
    rng = np.random.default_rng(5)
    A = rng.uniform(-1.0, 1.0, size=(1024, 1024))
    k = np.linalg.cond(A, 1)
    assert 4.4e4 < k < 4.4e8
