"""GPU tests of the runtime around the kernels: hipGraph replay of plans,
the autotuner and MP_AUTO, asynchronous LU, and the step profiler."""

import os
import tempfile

import numpy as np
import pytest

from helpers import first_mismatch, planes_equal
from oracle import cref
from paper_1410_1599_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1410_1599_amd import mp  # noqa: E402


def test_graph_replays_match_eager_and_oracle():
    p = 256
    m, l, n = 70, 90, 66
    s = torch.cuda.Stream()
    A0 = [I.uniform_pm1(m, l, p, 100 + r) for r in range(4)]
    B0 = [I.log_uniform(l, n, p, 200 + r, -10, 10) for r in range(4)]
    dA = mp.to_device(A0[0])
    dB = mp.to_device(B0[0])
    dC = mp.empty(m, n, p)
    mp.mp_set_graph_mode(True)
    try:
        with torch.cuda.stream(s):
            for r in range(4):
                # new operand values in the same buffers, eager torch work in between
                dA.copy_(mp.to_device(A0[r]))
                dB.copy_(mp.to_device(B0[r]))
                junk = torch.arange(1000, device="cuda").sum()
                mp.mp_gemm(m, l, n, p, mp.WINOGRAD, 8, dA, dB, dC)
                s.synchronize()
                got = mp.to_host(dC)
                want = cref.gemm(A0[r], B0[r], p, algo="winograd", cutoff=8)
                assert planes_equal(got, want), (r, first_mismatch(got, want, p))
                assert int(junk) == 499500
    finally:
        mp.mp_set_graph_mode(False)


@pytest.mark.parametrize("tcl,persist", [(0, 1), (5, 0), (5, 1), (4, 0), (4, 1)])
def test_launch_shapes_give_the_same_bits(tcl, persist):
    """Leaf tile width and persistent grids change no result bit: a ragged
    Winograd product (peels at every level, border tasks, many tiles) and a
    Block product against the default launch and the oracle."""
    p = 256
    m, l, n = 203, 150, 177
    A = I.uniform_pm1(m, l, p, 61)
    B = I.log_uniform(l, n, p, 62, -12, 12)
    dA, dB = mp.to_device(A), mp.to_device(B)
    ref, got = mp.empty(m, n, p), mp.empty(m, n, p)
    refb, gotb = mp.empty(m, n, p), mp.empty(m, n, p)
    mp.mp_gemm(m, l, n, p, mp.WINOGRAD, 16, dA, dB, ref)
    mp.mp_gemm(m, l, n, p, mp.BLOCK, 0, dA, dB, refb)
    mp.mp_set_launch(tcl, persist)
    try:
        mp.mp_gemm(m, l, n, p, mp.WINOGRAD, 16, dA, dB, got)
        mp.mp_gemm(m, l, n, p, mp.BLOCK, 0, dA, dB, gotb)
    finally:
        mp.mp_set_launch(0, 0)
    torch.cuda.synchronize()
    assert torch.equal(ref, got) and torch.equal(refb, gotb)
    want = cref.gemm(A, B, p, algo="winograd", cutoff=16)
    assert planes_equal(mp.to_host(got), want)


def test_launch_settings_rejected():
    with pytest.raises(mp.MPError):
        mp.mp_set_launch(3, 0)
    with pytest.raises(mp.MPError):
        mp.mp_set_launch(0, 2)


def test_tuner_and_auto_choice_reproducible():
    p = 256
    m, l, n = 130, 96, 140
    choice = mp.mp_tune(m, l, n, p, reps=1)
    assert choice["algo"] in (0, 1, 2, 3) and choice["ms"] > 0
    assert mp.mp_auto_choice(m, l, n, p) == {k: choice[k] for k in ("algo", "cutoff", "leaf")}
    launch = mp.mp_auto_launch(m, l, n, p)
    assert {k: launch[k] for k in ("algo", "cutoff", "leaf")} == mp.mp_auto_choice(m, l, n, p)
    assert launch["tile_cols_log2"] in (0, 4, 5) and launch["persistent"] in (0, 1)
    A = I.uniform_pm1(m, l, p, 7)
    B = I.uniform_pm1(l, n, p, 8)
    dA, dB = mp.to_device(A), mp.to_device(B)
    dC1, dC2 = mp.empty(m, n, p), mp.empty(m, n, p)
    mp.mp_gemm(m, l, n, p, mp.AUTO, 0, dA, dB, dC1)
    mp.mp_gemm_ex(m, l, n, p, choice["algo"], max(choice["cutoff"], 1), mp.PEEL, choice["leaf"], dA, dB, dC2)
    torch.cuda.synchronize()
    r1, r2 = mp.to_host(dC1), mp.to_host(dC2)
    assert planes_equal(r1, r2)
    names = {0: "simple", 1: "block", 2: "strassen", 3: "winograd"}
    want = cref.gemm(A, B, p, algo=names[choice["algo"]], cutoff=max(choice["cutoff"], 1))
    assert planes_equal(r1, want)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.json")
        mp.mp_tune_save(path)
        assert mp.mp_tune_load(path) >= 1
        assert mp.mp_auto_launch(m, l, n, p) == launch


def test_lu_async_matches_lu_ex():
    p, n = 256, 100
    A = I.uniform_pm1(n, n, p, 9)
    s = torch.cuda.Stream()
    dA1, dA2 = mp.to_device(A), mp.to_device(A)
    piv1 = torch.zeros(n, dtype=torch.int32, device="cuda")
    piv2 = torch.zeros(n, dtype=torch.int32, device="cuda")
    info_dev = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    info = mp.mp_lu_ex(n, p, dA1, piv1, 32, mp.WINOGRAD, 8)
    with torch.cuda.stream(s):
        mp.mp_lu_async(n, p, dA2, piv2, info_dev, 32, mp.WINOGRAD, 8)
    s.synchronize()
    assert info == 0 and int(info_dev.item()) == 0
    assert torch.equal(piv1, piv2)
    assert planes_equal(mp.to_host(dA1), mp.to_host(dA2))
    Fc, pc, ic = cref.lu(A, p, panel=32, algo="winograd", cutoff=8)
    assert planes_equal(mp.to_host(dA2), Fc) and list(piv2.cpu().numpy()) == list(pc)


def test_profiler_records_each_launch():
    p = 128
    A = mp.to_device(I.uniform_pm1(64, 64, p, 1))
    B = mp.to_device(I.uniform_pm1(64, 64, p, 2))
    C = mp.empty(64, 64, p)
    torch.cuda.synchronize()
    mp.mp_profile_read()
    mp.mp_profile(True)
    mp.mp_gemm(64, 64, 64, p, mp.WINOGRAD, 16, A, B, C)
    mp.mp_profile(False)
    recs = mp.mp_profile_read()
    info = mp.mp_plan_info(64, 64, 64, p, mp.WINOGRAD, 16)
    assert len(recs) == info["n_launches"]
    leaf = [r for r in recs if r["kind"] == 0]
    assert len(leaf) == 1 and leaf[0]["units"] == info["n_mul"] and leaf[0]["ms"] > 0
