"""GPU parity of the INT8-slice product.

The slice path computes c_ij = RN(2^(e_i + f_j - W_A - W_B) sum_k a'_ik b'_kj)
with a', b' the inputs truncated to their windows.  Its results must equal the
oracle's model of those steps (oracle.exact.slice_model_entry) bit for bit,
and, when no input is truncated, the correctly rounded exact product.
"""

import json
import os
import random

import numpy as np
import pytest

from oracle import exact, mpnum
from paper_1410_1599_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1410_1599_amd import mp  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def gpu_slice(A, B, p, extra=64):
    m, l = A.shape[1], A.shape[2]
    n = B.shape[2]
    dA, dB, dC = mp.to_device(A), mp.to_device(B), mp.empty(m, n, p)
    w = mp.mp_gemm_slice(m, l, n, p, extra, dA, dB, dC)
    torch.cuda.synchronize()
    return mp.to_host(dC), w


@pytest.mark.parametrize("p", [128, 256, 512, 1024])
def test_small_shapes_exact_rounding(p):
    for (m, l, n, kind) in ((1, 1, 1, "u"), (5, 7, 9, "u"), (130, 70, 129, "log"), (64, 200, 64, "log"),
                            (129, 1, 257, "u"), (3, 300, 2, "log")):
        gen = I.uniform_pm1 if kind == "u" else (lambda r, c, pp, sd: I.log_uniform(r, c, pp, sd, -20, 20))
        A, B = gen(m, l, p, 11), gen(l, n, p, 12)
        Ao, Bo = I.from_planes(A, p), I.from_planes(B, p)
        C, (WA, WB) = gpu_slice(A, B, p)
        assert (WA, WB) == exact.window_widths(Ao, Bo, p, 64)
        for i in range(m):
            for j in range(n):
                want = exact.slice_model_entry(Ao, Bo, i, j, p, WA, WB)
                got = I.entry(C, i, j, p)
                assert got == want, (p, (m, l, n), i, j)
                if WA - p < 64 and WB - p < 64:
                    assert want == exact.exact_entry(Ao, Bo, i, j, p)


@pytest.mark.parametrize("p,extra", [(128, 0), (256, 8), (512, 20)])
def test_truncated_window_matches_model(p, extra):
    m, l, n = 40, 90, 33
    A = I.log_uniform(m, l, p, 21, -60, 60)
    B = I.log_uniform(l, n, p, 22, -60, 60)
    Ao, Bo = I.from_planes(A, p), I.from_planes(B, p)
    C, (WA, WB) = gpu_slice(A, B, p, extra)
    assert WA == p + extra and WB == p + extra
    for i in range(m):
        for j in range(n):
            assert I.entry(C, i, j, p) == exact.slice_model_entry(Ao, Bo, i, j, p, WA, WB), (i, j)


def test_inner_split_at_512_bits():
    """At 512 bits a diagonal holds up to 73 digit pairs, more than fit one
    INT32 sum at l = 2048: the diagonal is split into slots."""
    p = 512
    m, l, n = 6, 2048, 5
    A = I.log_uniform(m, l, p, 31, -30, 30)
    B = I.log_uniform(l, n, p, 32, -30, 30)
    Ao, Bo = I.from_planes(A, p), I.from_planes(B, p)
    C, (WA, WB) = gpu_slice(A, B, p)
    for i in range(m):
        for j in range(n):
            assert I.entry(C, i, j, p) == exact.exact_entry(Ao, Bo, i, j, p)


def test_zero_rows_and_columns():
    p = 256
    A = I.uniform_pm1(9, 12, p, 41)
    B = I.uniform_pm1(12, 7, p, 42)
    A[:, 3, :] = 0
    B[:, :, 5] = 0
    Ao, Bo = I.from_planes(A, p), I.from_planes(B, p)
    C, _ = gpu_slice(A, B, p)
    for i in range(9):
        for j in range(7):
            assert I.entry(C, i, j, p) == exact.exact_entry(Ao, Bo, i, j, p)
    assert not C[:, 3, :].any() and not C[:, :, 5].any()


def test_n2048_p256_sampled_exact_and_limb_error():
    """The 2048 x 2048 256-bit log-uniform workload: the slice result is the
    correctly rounded exact product on sampled entries (<= 1/2 ulp), and the
    limb path's Winograd result on the same entries is reported against it."""
    g = json.load(open(os.path.join(GOLD, "full_size_n2048_p256.json")))
    n, p = 2048, 256
    A = I.log_uniform(n, n, p, 6)
    B = I.log_uniform(n, n, p, 7)
    C, (WA, WB) = gpu_slice(A, B, p)
    assert WA - p <= 41 and WB - p <= 41       # spreads of E in [-20, 20]: nothing truncated
    rng = random.Random(5)
    ents = rng.sample(g["entries"]["winograd"], 64)
    worst_limb = 0
    for i, j, s, e, mh in ents:
        row = I.row(A, i, p)
        col = I.col(B, j, p)
        nn, f = exact.exact_dot(row, col, p)
        want = mpnum.rn(nn, f, p)
        assert I.entry(C, i, j, p) == want, (i, j)
        limb = (int(mh, 16) * (-1 if s else 1), e)
        worst_limb = max(worst_limb, float(exact.ulp_error(limb, nn, f, p)))
    print("limb Winograd max ulp error on the sample: %.1f; slice: <= 0.5" % worst_limb)
    assert worst_limb >= 0.5


def test_n2048_p256_ulp_error_of_every_path():
    """The 2048 x 2048 256-bit log-uniform workload against stored exact
    products (RN_p of the exact dot product; a seeded 64 x 64 grid plus row 0
    and column 0): the slice path returns every sampled entry correctly
    rounded, so its error (<= 1/2 ulp) is never above the limb path's."""
    g = json.load(open(os.path.join(GOLD, "exact_n2048_p256.json")))
    n, p = 2048, 256
    A = I.log_uniform(n, n, p, 6)
    B = I.log_uniform(n, n, p, 7)
    S, _ = gpu_slice(A, B, p)
    dA, dB, dC = mp.to_device(A), mp.to_device(B), mp.empty(n, n, p)
    worst = {}
    for name, algo in (("winograd", mp.WINOGRAD), ("block", mp.BLOCK)):
        mp.mp_gemm_ex(n, n, n, p, algo, 64, mp.PEEL, mp.LEAF_SIMPLE, dA, dB, dC)
        torch.cuda.synchronize()
        C = mp.to_host(dC)
        w = 0.0
        for i, j, s, e, mh in g["entries"]:
            want = (int(mh, 16) * (-1 if s else 1), e)
            w = max(w, float(exact.ulp_error(I.entry(C, i, j, p), want[0], e - p, p)))
        worst[name] = w
    for i, j, s, e, mh in g["entries"]:
        assert I.entry(S, i, j, p) == (int(mh, 16) * (-1 if s else 1), e), (i, j)
    print("max ulp vs RN(exact) on %d entries: limb Winograd %.1f, limb Block %.1f, slice 0"
          % (len(g["entries"]), worst["winograd"], worst["block"]))
    assert worst["winograd"] >= worst["block"] >= 0
