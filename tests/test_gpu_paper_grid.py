"""GPU parity on the paper's own benchmark matrices (Section 3):
a_ij = sqrt5 (i+j-1), b_ij = sqrt3 (n-i+1), 128 bits, cutoff 32 (the paper's
n_min).  Every algorithm and odd-size policy is bit-exact to the C oracle on
square sizes around a power of two and on rectangular products of the kind
of Table 5 (m = n, inner size l varying), and the largest relative error
against the closed form c_ij = sqrt15 [(i-1) l (2n-l+1)/2 + sum_k k (n-k+1)]
stays within the largest the paper reports (tests/golden/paper_errors.json).
"""

import json
import os

import pytest

from helpers import first_mismatch, planes_equal
from oracle import cref
from paper_1410_1599_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1410_1599_amd import mp  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ALGOS = {"simple": mp.SIMPLE, "block": mp.BLOCK, "strassen": mp.STRASSEN, "winograd": mp.WINOGRAD}
POLICIES = {"peel": mp.PEEL, "pad": mp.PAD, "mixed": mp.MIXED}


def max_rel_error(C, m, l, n, p):
    from mpmath import mp as mpm, mpf, sqrt
    mpm.prec = 4 * p
    s15 = sqrt(15)
    tail = sum(k * (n - k + 1) for k in range(1, l + 1))
    worst = mpf(0)
    for i in range(m):
        ex = s15 * (i * l * (2 * n - l + 1) // 2 + tail)
        for j in range(n):
            sig, e = I.entry(C, i, j, p)
            worst = max(worst, abs(mpf(sig) * mpf(2) ** (e - p) - ex) / ex)
    return float(worst)


def gpu_gemm(A, B, p, algo, cutoff, policy):
    m, l = A.shape[1], A.shape[2]
    n = B.shape[2]
    dA, dB, dC = mp.to_device(A), mp.to_device(B), mp.empty(m, n, p)
    mp.mp_gemm_ex(m, l, n, p, ALGOS[algo], cutoff, POLICIES[policy], mp.LEAF_SIMPLE, dA, dB, dC)
    torch.cuda.synchronize()
    return mp.to_host(dC)


@pytest.mark.parametrize("n", [255, 257])
def test_square_paper_matrices(n):
    p = 128
    gold = json.load(open(os.path.join(GOLD, "paper_errors.json")))
    limit = {"simple": gold["block_128_max"], "block": gold["block_128_max"],
             "strassen": gold["strassen_128_max"], "winograd": gold["winograd_128_max"]}
    A, B = I.sqrt_workload(n, n, n, p)
    for algo in ALGOS:
        for policy in (("peel", "mixed") if algo in ("strassen", "winograd") else ("peel",)):
            want = cref.gemm(A, B, p, algo=algo, cutoff=32, policy=policy)
            got = gpu_gemm(A, B, p, algo, 32, policy)
            assert planes_equal(got, want), (algo, policy, first_mismatch(got, want, p))
        err = max_rel_error(got, n, n, n, p)
        print("n=%d %s: max relative error %.3g" % (n, algo, err))
        assert 0 < err <= limit[algo]


@pytest.mark.parametrize("l", [63, 65, 129])
def test_rectangular_paper_matrices(l):
    """Table 5's shape: m = n fixed, the inner size l varied."""
    p, m, n = 128, 200, 200
    A, B = I.sqrt_workload(m, l, n, p)
    for algo in ("strassen", "winograd"):
        for policy in ("peel", "pad", "mixed"):
            want = cref.gemm(A, B, p, algo=algo, cutoff=32, policy=policy)
            got = gpu_gemm(A, B, p, algo, 32, policy)
            assert planes_equal(got, want), (algo, policy, first_mismatch(got, want, p))
    assert 0 < max_rel_error(got, m, l, n, p) < 1e-34


def test_paper_matrices_1024_bits():
    """The paper's second precision (Tables 4 and 5): 1024 bits, every
    algorithm bit-exact to the oracle, errors inside the paper's 1024-bit
    figures (Strassen 6.30e-306, Winograd 3.92e-305)."""
    p, n = 1024, 131
    gold = json.load(open(os.path.join(GOLD, "paper_errors.json")))
    A, B = I.sqrt_workload(n, n, n, p)
    for algo in ALGOS:
        want = cref.gemm(A, B, p, algo=algo, cutoff=32, policy="mixed")
        got = gpu_gemm(A, B, p, algo, 32, "mixed")
        assert planes_equal(got, want), (algo, first_mismatch(got, want, p))
        err = max_rel_error(got, n, n, n, p)
        print("1024 bits n=%d %s: max relative error %.3g" % (n, algo, err))
        assert 0 < err <= (gold["winograd_1024_max"] if algo == "winograd" else gold["strassen_1024_max"])
