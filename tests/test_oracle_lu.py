"""Pins of the oracle's blocked LU with partial pivoting and solve.

* exact factorisation: A = P^T L U built from few-bit dyadic L (unit lower,
  |l_ij| < 1 so every pivot is unique) and U, where no operation rounds at
  p = 128: the oracle must return exactly P, L and U;
* LAPACK (scipy.linalg.lu_factor) on the same matrix in double precision
  picks the same pivot rows on a well-separated random matrix;
* the solve agrees with the exact rational solution within a first-order
  bound, and the exact residual ||PA - LU|| / ||A|| is tiny;
* the C oracle twin equals the Python oracle bit for bit and its
  high-precision residual agrees with the exact one.
"""

import random
from fractions import Fraction

import numpy as np
import pytest

from oracle import lu as LU, mpnum, cref, gemm as G
from paper_1410_1599_amd import inputs as I


def dyadic(rng, bits, emin, emax):
    v = rng.randrange(1, 1 << bits)
    return Fraction(rng.choice((1, -1)) * v, 1 << rng.randint(-emin, -emin + (emax - emin)))


def exact_case(n, seed, p=128):
    """A = P^T L U with small dyadic factors; returns (A, P as list, L, U) as Fractions."""
    rng = random.Random(seed)
    L = [[Fraction(0)] * n for _ in range(n)]
    U = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        L[i][i] = Fraction(1)
        for j in range(i):
            # |l_ij| < 1: multiples of 1/16 in (-1, 1), distinct from +-1
            L[i][j] = Fraction(rng.randrange(-15, 16), 16)
        U[i][i] = Fraction(rng.choice((1, -1)) * rng.randrange(1, 16), 4)
        for j in range(i + 1, n):
            U[i][j] = Fraction(rng.randrange(-31, 32), 8)
    LUp = [[sum(L[i][k] * U[k][j] for k in range(n)) for j in range(n)] for i in range(n)]
    perm = list(range(n))
    rng.shuffle(perm)                       # A[perm[i]] = (LU)[i]
    A = [None] * n
    for i in range(n):
        A[perm[i]] = LUp[i]
    return A, perm, L, U


def to_mp(M, p):
    return [[mpnum.from_fraction(v, p) for v in row] for row in M]


@pytest.mark.parametrize("algo,panel,cutoff", [("winograd", 4, 1), ("strassen", 3, 1), ("simple", 5, 8), ("winograd", 16, 2)])
def test_exact_factorisation_recovered(algo, panel, cutoff):
    p = 128
    n = 13
    A, perm, L, U = exact_case(n, 5, p)
    Am = to_mp(A, p)
    F, piv, info = LU.lu(Am, p, panel=panel, algo=algo, cutoff=cutoff)
    assert info == 0
    # replay the swaps on the identity to get the row order
    order = list(range(n))
    for k, r in enumerate(piv):
        order[k], order[r] = order[r], order[k]
    assert order == perm
    for i in range(n):
        for j in range(n):
            v = mpnum.to_fraction(F[i][j], p)
            if j < i:
                assert v == L[i][j]
            else:
                assert v == U[i][j]


def test_pivots_match_lapack_on_random_matrix():
    from scipy.linalg import lu_factor
    p = 256
    n = 40
    rng = np.random.default_rng(12)
    D = rng.uniform(-1, 1, size=(n, n))
    A = [[mpnum.from_fraction(Fraction(float(D[i, j])), p) for j in range(n)] for i in range(n)]
    F, piv, info = LU.lu(A, p, panel=8, algo="winograd", cutoff=4)
    _, lp = lu_factor(D)
    assert list(piv) == [int(v) for v in lp]
    assert info == 0


def test_zero_pivot_reports_info():
    p = 128
    n = 6
    A = [[mpnum.from_int(1 if (i == j and i != 3) else 0, p) for j in range(n)] for i in range(n)]
    F, piv, info = LU.lu(A, p, panel=4)
    assert info == 4
    Ac = I.to_planes(A, p)
    F2, piv2, info2 = cref.lu(Ac, p, panel=4)
    assert info2 == 4 and list(piv2) == piv
    assert I.from_planes(F2, p) == F


def test_solve_and_residual_small():
    p = 128
    n = 12
    Ap = I.uniform_pm1(n, n, p, 33)
    A = I.from_planes(Ap, p)
    b = LU.rhs_ones(A, p)
    F, piv, info = LU.lu(A, p, panel=5, algo="winograd", cutoff=2)
    x = LU.solve(F, piv, b, p)
    # exact solution of A x = b (b as computed)
    Af = [[mpnum.to_fraction(v, p) for v in r] for r in A]
    bf = [mpnum.to_fraction(v, p) for v in b]
    xs = gauss_exact(Af, bf)
    err = max(abs(mpnum.to_fraction(x[i], p) - xs[i]) for i in range(n))
    assert err < Fraction(1, 1 << (p - 40))
    res = LU.residual_exact(A, F, piv, p)
    assert 0 < res < Fraction(n * n * 16, 1 << p)


def gauss_exact(A, b):
    n = len(A)
    M = [list(r) + [bb] for r, bb in zip(A, b)]
    for c in range(n):
        r = next(i for i in range(c, n) if M[i][c] != 0)
        M[c], M[r] = M[r], M[c]
        for i in range(n):
            if i != c and M[i][c] != 0:
                f = M[i][c] / M[c][c]
                M[i] = [a - f * bb for a, bb in zip(M[i], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


@pytest.mark.parametrize("p", [128, 512])
@pytest.mark.parametrize("kind", ["random", "hilbert"])
def test_c_oracle_lu_matches_python(p, kind):
    n = 19
    A = I.uniform_pm1(n, n, p, 8) if kind == "random" else I.hilbert(n, p)
    Ao = I.from_planes(A, p)
    for algo, panel, cut in (("winograd", 8, 2), ("strassen", 6, 1), ("simple", 7, 4)):
        Fp, pivp, infop = LU.lu(Ao, p, panel=panel, algo=algo, cutoff=cut)
        Fc, pivc, infoc = cref.lu(A, p, panel=panel, algo=algo, cutoff=cut)
        assert list(pivc) == pivp and infoc == infop
        assert I.from_planes(Fc, p) == Fp, (algo, panel)
        bp = LU.rhs_ones(Ao, p)
        xp = LU.solve(Fp, pivp, bp, p)
        bc = I.to_planes([[v] for v in bp], p)
        xc = cref.lu_solve(Fc, pivc, bc, p)
        assert [r[0] for r in I.from_planes(xc, p)] == xp


def test_c_residual_matches_exact():
    import math
    p = 128
    n = 14
    A = I.uniform_pm1(n, n, p, 9)
    Ao = I.from_planes(A, p)
    F, piv, info = cref.lu(A, p, panel=4, algo="winograd", cutoff=2)
    l2, val = cref.lu_residual(A, F, piv, p)
    ex = LU.residual_exact(Ao, I.from_planes(F, p), list(piv), p)
    assert ex > 0
    assert abs(l2 - math.log2(ex)) < 1e-6


@pytest.mark.parametrize("algo,panel,cutoff", [("winograd", 4, 1), ("strassen", 5, 1), ("simple", 13, 8)])
def test_unpivoted_exact_factorisation_recovered(algo, panel, cutoff):
    """The paper's LU without row exchanges (Section 4) on A = L U with small
    dyadic factors whose multipliers are not the largest in their columns
    (|l_ij| up to 4): nothing rounds, so the factors come back exactly, the
    pivots are the identity, and partial pivoting would have swapped."""
    p = 128
    n = 11
    rng = random.Random(9)
    L = [[Fraction(0)] * n for _ in range(n)]
    U = [[Fraction(0)] * n for _ in range(n)]
    for i in range(n):
        L[i][i] = Fraction(1)
        for j in range(i):
            L[i][j] = Fraction(rng.randrange(-63, 64), 16)
        U[i][i] = Fraction(rng.choice((1, -1)) * rng.randrange(1, 8), 8)
        for j in range(i + 1, n):
            U[i][j] = Fraction(rng.randrange(-31, 32), 8)
    A = [[sum(L[i][k] * U[k][j] for k in range(n)) for j in range(n)] for i in range(n)]
    Am = to_mp(A, p)
    F, piv, info = LU.lu(Am, p, panel=panel, algo=algo, cutoff=cutoff, pivot=False)
    assert info == 0 and piv == list(range(n))
    for i in range(n):
        for j in range(n):
            v = mpnum.to_fraction(F[i][j], p)
            assert v == (L[i][j] if j < i else U[i][j]), (i, j)
    _, pivp, _ = LU.lu(Am, p, panel=panel, algo=algo, cutoff=cutoff)
    assert pivp != list(range(n))


@pytest.mark.parametrize("p", [128, 512])
@pytest.mark.parametrize("kind", ["random", "lotkin"])
def test_c_oracle_unpivoted_lu_matches_python(p, kind):
    n = 17
    A = I.uniform_pm1(n, n, p, 8) if kind == "random" else I.lotkin(n, p)
    Ao = I.from_planes(A, p)
    for algo, panel, cut in (("winograd", 8, 2), ("simple", 5, 4)):
        Fp, pivp, infop = LU.lu(Ao, p, panel=panel, algo=algo, cutoff=cut, pivot=False)
        Fc, pivc, infoc = cref.lu(A, p, panel=panel, algo=algo, cutoff=cut, pivot=False)
        assert list(pivc) == pivp == list(range(n)) and infoc == infop == 0
        assert I.from_planes(Fc, p) == Fp, (algo, panel)


def test_unpivoted_lotkin_solve_close_to_arange():
    """x = [0, 1, ..., n-1] and b = A x for the Lotkin matrix (the paper's
    ill-conditioned case, Section 4): the unpivoted factors solve it to within
    the condition number (about 1e8 at n = 8) times the unit roundoff."""
    p, n = 256, 8
    A = I.lotkin(n, p)
    Ao = I.from_planes(A, p)
    x = I.from_planes(I.arange_column(n, p), p)
    b = [r[0] for r in G.gemm(Ao, x, p, algo=G.SIMPLE)]
    F, piv, info = LU.lu(Ao, p, panel=3, algo=G.WINOGRAD, cutoff=1, pivot=False)
    assert info == 0
    xs = LU.solve(F, piv, b, p)
    err = max(abs(mpnum.to_fraction(v, p) - i) for i, v in enumerate(xs))
    assert err < Fraction(1, 2 ** 200)


@pytest.mark.parametrize("p", [128, 1024])
def test_division_stress_matrix_pivots_and_multipliers(p):
    """The matrix that strains the GPU's lane division (tests/helpers.py): in the
    oracle's LU its first K pivots are the diagonal, and every multiplier
    l_ij (j < K) is the correctly rounded quotient of the entries as built
    (the zeros above the diagonal leave column j unchanged until its step);
    exchanges of later columns move whole rows, multipliers included."""
    from helpers import division_stress_matrix
    n, K = 70, 64
    A, top_equal = division_stress_matrix(p, n, K, 77 + p)
    assert top_equal > 300
    F, piv, info = cref.lu(A, p, panel=32, algo="simple", cutoff=8)
    assert info == 0 and list(piv[:K]) == list(range(K))
    row = list(range(n))
    for c in range(n):
        r = int(piv[c])
        row[c], row[r] = row[r], row[c]
    for j in range(K):
        y = I.entry(A, j, j, p)
        for i in range(j + 1, n):
            assert I.entry(F, i, j, p) == mpnum.div(I.entry(A, row[i], j, p), y, p), (i, j)
