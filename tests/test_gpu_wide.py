"""GPU parity at 2048, 4096, 8192 and 10240 bits (one value per wavefront), bit for
bit against the Python oracle:

* scalar mul/add/sub/div on adversarial operands (gaps around 0, 32, 64, p,
  ties, cancellation, gaps past the guard) and random ones;
* every algorithm and odd-size policy on ragged shapes at small cutoffs;
* LU with and without pivoting (Winograd trailing updates) and the solve;
* the paper's use of 8192 bits: the unpivoted LU of the Lotkin matrix
  (Section 4) with x = [0 .. n-1].
"""

import random
from fractions import Fraction

import numpy as np
import pytest

from helpers import adversarial_pairs, first_mismatch, planes_equal, random_value, vec_planes
from oracle import gemm as G, lu as LU, mpnum
from paper_1410_1599_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1410_1599_amd import mp  # noqa: E402

WIDE = [2048, 4096, 8192, 10240]


def sync():
    torch.cuda.synchronize()


@pytest.mark.parametrize("p", WIDE)
def test_wide_scalar_ops(p):
    rng = random.Random(700 + p)
    pairs = adversarial_pairs(rng, p) + [(random_value(rng, p, -40, 40), random_value(rng, p, -40, 40))
                                         for _ in range(300)]
    X = vec_planes([x for x, _ in pairs], p)
    Y = vec_planes([y for _, y in pairs], p)
    dX, dY = mp.to_device(X), mp.to_device(Y)
    N = len(pairs)
    print("p", p, "pairs", N, flush=True)
    for name, fn, ref in (("mul", mp.mp_mul_ew, mpnum.mul), ("add", mp.mp_add, mpnum.add),
                          ("sub", mp.mp_sub, mpnum.sub), ("div", mp.mp_div_ew, mpnum.div)):
        keep = [k for k, (_, y) in enumerate(pairs) if y[0] != 0] if name == "div" else range(N)
        dZ = mp.empty(1, N, p)
        fn(1, N, p, dX, dY, dZ)
        sync()
        Z = mp.to_host(dZ)
        for k in keep:
            x, y = pairs[k]
            assert I.entry(Z, 0, k, p) == ref(x, y, p), (name, p, x, y)


@pytest.mark.parametrize("p", WIDE)
def test_wide_division_digit_estimate(p):
    """Divisors with long runs of ones or zeros below the top limbs, and
    quotients near 1, stress the radix-2^32 digit estimate and its corrections."""
    rng = random.Random(950 + p)
    one = 1 << (p - 1)
    pairs = [(random_value(rng, p, -300, 300), random_value(rng, p, -300, 300)) for _ in range(300)]
    for _ in range(150):
        run = rng.randrange(1, p)
        pairs.append(((rng.randrange(one, 1 << p), 0), (((1 << p) - 1) ^ ((1 << run) - 1) | one, 0)))
        pairs.append(((rng.randrange(one, 1 << p), 0), (one | ((1 << run) - 1), 0)))
        pairs.append((((1 << p) - 1 - rng.randrange(0, 1 << 16), 0), (one + rng.randrange(0, 1 << 16), 0)))
        m = rng.randrange(one, 1 << p)
        pairs.append(((m, 3), (m, 1)))
        pairs.append(((m, 0), (m + 1 if m + 1 < (1 << p) else m - 1, 0)))
    X = vec_planes([x for x, _ in pairs], p)
    Y = vec_planes([y for _, y in pairs], p)
    dZ = mp.empty(1, len(pairs), p)
    mp.mp_div_ew(1, len(pairs), p, mp.to_device(X), mp.to_device(Y), dZ)
    sync()
    Z = mp.to_host(dZ)
    for k, (x, y) in enumerate(pairs):
        assert I.entry(Z, 0, k, p) == mpnum.div(x, y, p), (x, y)


@pytest.mark.parametrize("p", WIDE)
def test_wide_gemm_all_algorithms(p):
    rng = np.random.default_rng(p + 3)
    for (m, l, n) in ((1, 1, 1), (9, 9, 9), (17, 19, 18)):
        seed = int(rng.integers(0, 1 << 30))
        A = I.uniform_pm1(m, l, p, seed)
        B = I.log_uniform(l, n, p, seed + 1, -30, 30)
        Ao, Bo = I.from_planes(A, p), I.from_planes(B, p)
        for algo in ("simple", "block", "strassen", "winograd"):
            for policy in (("peel", "pad", "mixed") if algo in ("strassen", "winograd") else ("peel",)):
                cut = 4
                want = I.to_planes(G.gemm(Ao, Bo, p, algo=algo, cutoff=cut, policy=policy, block_size=16), p)
                dA, dB, dC = mp.to_device(A), mp.to_device(B), mp.empty(m, n, p)
                mp.mp_gemm_ex(m, l, n, p, mp.ALGOS[algo], cut, mp.POLICIES[policy], mp.LEAF_SIMPLE, dA, dB, dC)
                sync()
                got = mp.to_host(dC)
                assert planes_equal(got, want), (p, algo, policy, (m, l, n), first_mismatch(got, want, p))


def _gpu_lu(A, p, panel, algo, cutoff, pivot):
    n = A.shape[1]
    dA = mp.to_device(A)
    piv = torch.zeros(n, dtype=torch.int32, device="cuda")
    f = mp.mp_lu_ex if pivot else mp.mp_lu_nopivot
    info = f(n, p, dA, piv, panel, algo, cutoff, mp.PEEL)
    sync()
    return mp.to_host(dA), piv.cpu().numpy(), info


def _gpu_solve(F, piv, b, p):
    n = F.shape[1]
    db = mp.to_device(b)
    mp.mp_lu_solve(n, p, mp.to_device(F), torch.from_numpy(np.ascontiguousarray(piv, dtype=np.int32)).cuda(), db)
    sync()
    return mp.to_host(db)


@pytest.mark.parametrize("p", [2048, 8192, 10240])
@pytest.mark.parametrize("pivot", [True, False])
def test_wide_lu_and_solve(p, pivot):
    n, panel, cut = 13, 5, 2
    A = I.uniform_pm1(n, n, p, 17)
    Ao = I.from_planes(A, p)
    Fo, po, io = LU.lu(Ao, p, panel=panel, algo=G.WINOGRAD, cutoff=cut, pivot=pivot)
    Fg, pg, ig = _gpu_lu(A, p, panel, mp.WINOGRAD, cut, pivot)
    assert ig == io and list(pg) == list(po)
    assert planes_equal(Fg, I.to_planes(Fo, p)), first_mismatch(Fg, I.to_planes(Fo, p), p)
    b = LU.rhs_ones(Ao, p)
    xo = LU.solve(Fo, po, b, p)
    bp = I.to_planes([[v] for v in b], p)
    assert planes_equal(_gpu_solve(Fg, pg, bp, p), I.to_planes([[v] for v in xo], p))


def test_wide_lotkin_8192_unpivoted():
    """The paper's ill-conditioned case at its precision (Section 4): the
    Lotkin matrix, x = [0 .. n-1], b = A x by Simple, LU without pivoting,
    Winograd trailing updates; factors and solution equal the oracle's, and
    the solution is x to within the condition number times 2^-8192."""
    p, n = 8192, 24
    A = I.lotkin(n, p)
    x = I.arange_column(n, p)
    Ao = I.from_planes(A, p)
    Fo, po, io = LU.lu(Ao, p, panel=8, algo=G.WINOGRAD, cutoff=2, pivot=False)
    Fg, pg, ig = _gpu_lu(A, p, 8, mp.WINOGRAD, 2, False)
    assert ig == io == 0
    assert planes_equal(Fg, I.to_planes(Fo, p)), first_mismatch(Fg, I.to_planes(Fo, p), p)
    b = G.gemm(Ao, I.from_planes(x, p), p, algo=G.SIMPLE)
    xo = LU.solve(Fo, po, [r[0] for r in b], p)
    xg = _gpu_solve(Fg, pg, I.to_planes(b, p), p)
    assert planes_equal(xg, I.to_planes([[v] for v in xo], p))
    tol = Fraction(1, 1 << 7000)
    for i in range(n):
        v = mpnum.to_fraction(I.entry(xg, i, 0, p), p)
        assert abs(v - i) < tol, i


def test_wide_precisions_refused_where_unsupported():
    """The INT8-slice product and the device fill exist up to 1024 bits only:
    they refuse wider precisions with MP_E_PREC and launch nothing."""
    p = 2048
    A = mp.to_device(I.uniform_pm1(3, 3, p, 1))
    C = mp.empty(3, 3, p)
    with pytest.raises(mp.MPError) as e:
        mp.mp_gemm_slice(3, 3, 3, p, 64, A, A, C)
    assert e.value.code == -2
    with pytest.raises(mp.MPError) as e:
        mp.mp_fill_uniform(3, 3, p, C, 1)
    assert e.value.code == -2
    assert not mp.to_host(C).any()
