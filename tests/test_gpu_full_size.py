"""GPU parity at the full workload sizes, in the launch configuration bench.py
times (mp_gemm_ex, peel, Simple leaves), on sampled entries.

Strassen and Winograd are compared with entries the C oracle computed once
for the same seeded inputs (tests/golden/make_full_size.py); Simple and Block
are compared with rows the C oracle computes here (Simple's rows are
independent, and Block is bit-identical to Simple).
"""

import json
import os

import numpy as np
import pytest

from helpers import first_mismatch, planes_equal
from oracle import cref
from paper_1410_1599_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1410_1599_amd import mp  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def inputs_for(g):
    n, p = g["n"], g["p"]
    gen = I.uniform_pm1 if g["kind"] == "uniform" else I.log_uniform
    return gen(n, n, p, g["seeds"][0]), gen(n, n, p, g["seeds"][1])


def gpu_product(A, B, p, algo, cutoff):
    n = A.shape[1]
    dA, dB, dC = mp.to_device(A), mp.to_device(B), mp.empty(n, n, p)
    mp.mp_gemm_ex(n, n, n, p, algo, cutoff, mp.PEEL, mp.LEAF_SIMPLE, dA, dB, dC)
    torch.cuda.synchronize()
    return mp.to_host(dC)


@pytest.mark.parametrize("name", ["full_size_n1023_p256", "full_size_n1024_p256", "full_size_n2048_p256"])
def test_fast_algorithms_sampled_entries(name):
    path = os.path.join(GOLD, name + ".json")
    g = json.load(open(path))
    A, B = inputs_for(g)
    p = g["p"]
    for algo, ents in g["entries"].items():
        C = gpu_product(A, B, p, mp.ALGOS[algo], g["cutoff"])
        bad = []
        for i, j, s, e, mh in ents:
            want = (int(mh, 16) * (-1 if s else 1), e)
            got = I.entry(C, i, j, p)
            if got != want:
                bad.append((i, j, got, want))
        assert not bad, (name, algo, len(bad), bad[:3])


@pytest.mark.parametrize("n,kind", [(1023, "uniform"), (2048, "log_uniform")])
def test_simple_and_block_sampled_rows(n, kind):
    p = 256
    seeds = (3, 4) if kind == "uniform" else (6, 7)
    gen = I.uniform_pm1 if kind == "uniform" else I.log_uniform
    A, B = gen(n, n, p, seeds[0]), gen(n, n, p, seeds[1])
    rows = [0, 1, n // 2, n - 1]
    want = cref.gemm(np.ascontiguousarray(A[:, rows, :]), B, p, algo="simple", m=len(rows))
    for algo in (mp.SIMPLE, mp.BLOCK):
        C = gpu_product(A, B, p, algo, 0)
        got = np.ascontiguousarray(C[:, rows, :])
        assert planes_equal(got, want), (algo, first_mismatch(got, want, p))
