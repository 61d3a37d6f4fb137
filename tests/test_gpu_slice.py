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


# ------------------------------------------------------------------ early stop

def _slice_guard(A, B, p, guard):
    mp.mp_set_slice_guard(guard)
    try:
        C, w = gpu_slice(A, B, p)
        info = mp.mp_slice_last()
    finally:
        mp.mp_set_slice_guard(32)
    return C, w, info


@pytest.mark.parametrize("p", [128, 256, 512, 1024])
def test_early_stop_equals_one_pass(p):
    """The two-pass product (diagonals u >= u0 first, low diagonals only for
    undecided tiles) equals the one-pass product bit for bit, with the default
    guard and with guard 0 (almost every tile recomputed)."""
    for (m, l, n, kind, seed) in ((300, 96, 290, "log", 51), (257, 64, 513, "u", 53)):
        gen = I.uniform_pm1 if kind == "u" else (lambda r, c, pp, sd: I.log_uniform(r, c, pp, sd, -20, 20))
        A, B = gen(m, l, p, seed), gen(l, n, p, seed + 1)
        C0, w0, info0 = _slice_guard(A, B, p, -1)
        assert info0[0] == 0
        for guard in (32, 0):
            C1, w1, info1 = _slice_guard(A, B, p, guard)
            assert w1 == w0
            assert info1[0] > 0 and info1[1] == info0[1], info1
            assert np.array_equal(C1, C0), (p, (m, l, n), guard, info1)
        print("p", p, (m, l, n), "guard 0 recomputed", info1[2], "of", info1[3], "tiles")


def test_early_stop_recomputes_cancelling_tiles():
    """Sums that cancel exactly or nearly are undecided after the first pass:
    their tiles are recomputed from every diagonal and come out correctly
    rounded (exact zeros as +0); the other tiles are decided at once."""
    p, L = 256, 8
    m, l, n, h = 260, 64, 520, 32
    A = I.uniform_pm1(m, l, p, 61)
    B = I.uniform_pm1(l, n, p, 62)
    A[:, :, h:] = A[:, :, :h]
    # columns 256.. : b_(k+h) = -b_k, so c_ij = 0; odd columns get the last
    # bit of one entry flipped, so c_ij = +-a_i,l-1 * ulp(b): tiny and nonzero
    for j in range(256, n):
        B[:, h:, j] = B[:, :h, j]
        nz = B[L - 1, h:, j] != 0
        B[L + 1, h:, j] = np.where(nz, B[L + 1, h:, j] ^ 1, 0)
        if j % 2:
            B[0, l - 1, j] ^= 1
    C, _, info = _slice_guard(A, B, p, 32)
    assert info[0] > 0
    assert info[2] == 4 and info[3] == 6, info    # 2 row tiles x column tiles 1, 2
    C0, _, _ = _slice_guard(A, B, p, -1)
    assert np.array_equal(C, C0)
    Ao, Bo = I.from_planes(A, p), I.from_planes(B, p)
    for i in (0, 129, 259):
        for j in list(range(0, 8)) + list(range(250, 270)) + list(range(510, 520)):
            assert I.entry(C, i, j, p) == exact.exact_entry(Ao, Bo, i, j, p), (i, j)
    zero_cols = [j for j in range(256, n) if j % 2 == 0]
    assert not C[:, :, zero_cols].any()
    assert C[:L, :, [j for j in range(257, n, 2)]].any(axis=0).all()


def test_early_stop_guard_settings():
    p = 256
    A = I.log_uniform(70, 80, p, 71, -20, 20)
    B = I.log_uniform(80, 60, p, 72, -20, 20)
    _, _, info = _slice_guard(A, B, p, 1 << 20)
    assert info[0] == 0
    _, _, info = _slice_guard(A, B, p, 32)
    assert 0 < info[0] < info[1] and info[4] > 0
    with pytest.raises(RuntimeError):
        mp.mp_set_slice_guard((1 << 20) + 1)
