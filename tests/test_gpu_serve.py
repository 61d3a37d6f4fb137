"""GPU test of the request loop: every request completes, results of a
sample equal the same requests run alone (bit for bit), and a product and a
solve from the mix equal the CPU oracle on the same device-generated operands."""

import numpy as np
import pytest

from helpers import planes_equal
from oracle import cref
from paper_1410_1599_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1410_1599_amd import mp, serve  # noqa: E402


def test_mix_completes_and_matches_alone_and_oracle():
    reqs = serve.make_requests(160, 4000.0, seed=21, gemm_range=(32, 300), lu_range=(64, 160))
    keep = {r.rid for r in reqs[::5]}
    srv = serve.Server(slots=4, keep=keep)
    st = srv.run(reqs)
    assert st["requests"] == 160 and all(r.t_done is not None and r.t_done >= r.arrival for r in reqs)
    assert st["p99_ms"] >= st["p50_ms"] > 0
    sample = [r for r in reqs if r.rid in keep]
    ref = srv.alone(sample)
    for r in sample:
        assert planes_equal(ref[r.rid], r.result), r.rid
    # one product and one solve against the oracle, same seeded device operands
    g = next(r for r in sample if r.kind == "gemm")
    m, l, n = g.dims
    A, B = mp.empty(m, l, g.prec), mp.empty(l, n, g.prec)
    mp.mp_fill_uniform(m, l, g.prec, A, g.seed)
    mp.mp_fill_uniform(l, n, g.prec, B, g.seed ^ 0x5555)
    torch.cuda.synchronize()
    want = cref.gemm(mp.to_host(A), mp.to_host(B), g.prec, algo="winograd", cutoff=64)
    assert planes_equal(g.result, want)
    lus = [r for r in reqs if r.kind == "lu"]
    if lus:
        r = lus[0]
        n, p = r.dims[0], r.prec
        A = mp.empty(n, n, p)
        mp.mp_fill_uniform(n, n, p, A, r.seed)
        torch.cuda.synchronize()
        Ah = mp.to_host(A)
        b = cref.gemm(Ah, I.ones_column(n, p), p, algo="simple")
        F, piv, info = cref.lu(Ah, p, panel=64, algo="winograd", cutoff=32)
        x = cref.lu_solve(F, piv, b, p)
        got = srv.alone([r])[r.rid]
        assert planes_equal(got, x)


def test_fill_uniform_values_in_range():
    p = 256
    X = mp.empty(40, 50, p)
    mp.mp_fill_uniform(40, 50, p, X, 123)
    torch.cuda.synchronize()
    h = mp.to_host(X)
    L = p // 32
    assert ((h[L - 1] >> 31) == 1).mean() > 0.99          # normalised mantissas
    e = h[L].view(np.int32)
    assert (e <= 0).all() and (e > -64).all()              # |x| < 1


def test_binding_budget_refuses_queues_and_matches_alone():
    """A 0.3 GB budget binds on this mix: the requests whose footprint alone
    exceeds it are refused (never launched), others wait for memory to free
    up, admitted memory never exceeds the budget, and results are the same
    bits as the same requests run alone."""
    reqs = serve.make_requests(120, 3000.0, seed=22)
    budget = 0.3 * 2 ** 30
    keep = {r.rid for r in reqs[::3]}
    srv = serve.Server(slots=4, hbm_budget_gb=0.3, keep=keep)
    st = srv.run(reqs)
    want_refused = {r.rid for r in reqs if serve.footprint(r) > budget}
    assert len(want_refused) >= 2
    assert {r.rid for r in reqs if r.status == serve.REFUSED} == want_refused
    assert all(r.status == serve.OK for r in reqs if r.rid not in want_refused)
    assert st["waited_for_memory"] > 0
    assert st["peak_admitted_gb"] <= 0.3
    sample = [r for r in reqs if r.rid in keep and r.status == serve.OK]
    ref = srv.alone(sample)
    for r in sample:
        assert planes_equal(ref[r.rid], r.result), r.rid
