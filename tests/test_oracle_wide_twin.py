"""The C oracle's wide build (up to 656 limbs: 10240-bit values and their
2p + 64-bit residuals) against the Python oracle at 2048, 8192 and 10240
bits: scalar operations on adversarial pairs, every algorithm and odd-size
policy on ragged shapes, LU with and without pivoting and the solve.  The
wide build is what writes the expected values of the GPU tests at those
precisions, so it is pinned here first (CPU only)."""

import random

import pytest

from helpers import adversarial_pairs, random_value
from oracle import cref, gemm as G, lu as LU, mpnum
from paper_1410_1599_amd import inputs as I

WIDE = [2048, 8192, 10240]


def rec(v, p):
    a = I.empty(1, 1, p)
    I.set_entry(a, 0, 0, v, p)
    return a.reshape(-1).copy()


def unrec(r, p):
    return I.entry(r.reshape(p // 32 + 2, 1, 1), 0, 0, p)


@pytest.mark.parametrize("p", WIDE)
def test_wide_twin_scalar_matches_python(p):
    rng = random.Random(91 + p)
    pairs = adversarial_pairs(rng, p)
    pairs = rng.sample(pairs, 120) + [(random_value(rng, p), random_value(rng, p)) for _ in range(40)]
    for x, y in pairs:
        for op, f in (("mul", mpnum.mul), ("add", mpnum.add), ("sub", mpnum.sub), ("div", mpnum.div)):
            if op == "div" and (y[0] == 0 or rng.random() < 0.7):
                continue                      # the twin's division is bit-serial: a sample suffices
            got = unrec(cref.scalar(op, p, rec(x, p), rec(y, p)), p)
            assert got == f(x, y, p), (op, x, y)


@pytest.mark.parametrize("p", WIDE)
def test_wide_twin_gemm_matches_python(p):
    for (m, l, n, cut, seed) in ((7, 6, 9, 2, 1), (8, 8, 8, 1, 2), (5, 9, 4, 2, 3)):
        A = I.uniform_pm1(m, l, p, seed)
        B = I.log_uniform(l, n, p, seed + 50, -5, 5)
        Ao, Bo = I.from_planes(A, p), I.from_planes(B, p)
        for algo in ("simple", "strassen", "winograd"):
            for policy in (("peel", "pad", "mixed") if algo != "simple" else ("peel",)):
                Cp = G.gemm(Ao, Bo, p, algo=algo, cutoff=cut, policy=policy)
                Cc = I.from_planes(cref.gemm(A, B, p, algo=algo, cutoff=cut, policy=policy), p)
                assert Cp == Cc, (algo, policy, m, l, n)


@pytest.mark.parametrize("p", [2048, 10240])
@pytest.mark.parametrize("pivot", [True, False])
def test_wide_twin_lu_and_solve_match_python(p, pivot):
    n = 9
    A = I.uniform_pm1(n, n, p, 8) if pivot else I.lotkin(n, p)
    Ao = I.from_planes(A, p)
    Fp, pivp, infop = LU.lu(Ao, p, panel=4, algo="winograd", cutoff=1, pivot=pivot)
    Fc, pivc, infoc = cref.lu(A, p, panel=4, algo="winograd", cutoff=1, pivot=pivot)
    assert list(pivc) == pivp and infoc == infop
    assert I.from_planes(Fc, p) == Fp
    bp = LU.rhs_ones(Ao, p)
    xp = LU.solve(Fp, pivp, bp, p)
    xc = cref.lu_solve(Fc, pivc, I.to_planes([[v] for v in bp], p), p)
    assert [r[0] for r in I.from_planes(xc, p)] == xp
    l2, _ = cref.lu_residual(A, Fc, pivc, p)
    assert l2 < -p + 16
