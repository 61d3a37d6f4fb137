"""GPU parity at the full workload sizes, in the launch configuration bench.py
times (mp_gemm_ex, peel, Simple leaves), on the whole result.

Every product is compared with the sha256 of the C oracle's complete result
for the same seeded inputs, algorithm and cutoff (written once by
tests/golden/make_full_size.py, which calls only the oracle): n = 1023 and
1024 at 256 bits with all four algorithms, and the 2048 x 2048 log-uniform
product with Winograd, Strassen, Simple and Block (Block against Simple's
digest: the two are bit-identical, an oracle invariant pinned on the CPU).
On a mismatch the stored sampled entries name the first differing ones.
"""

import hashlib
import json
import os

import numpy as np
import pytest

from paper_1410_1599_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1410_1599_amd import mp  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden")
_inputs = {}


def golden(name):
    return json.load(open(os.path.join(GOLD, name + ".json")))


def device_inputs(g):
    key = (g["n"], g["p"], g["kind"], tuple(g["seeds"]))
    if key not in _inputs:
        _inputs.clear()
        n, p = g["n"], g["p"]
        gen = I.uniform_pm1 if g["kind"] == "uniform" else I.log_uniform
        _inputs[key] = (mp.to_device(gen(n, n, p, g["seeds"][0])), mp.to_device(gen(n, n, p, g["seeds"][1])))
    return _inputs[key]


def gpu_product(g, algo, leaf=mp.LEAF_SIMPLE):
    n, p = g["n"], g["p"]
    dA, dB = device_inputs(g)
    dC = mp.empty(n, n, p)
    mp.mp_gemm_ex(n, n, n, p, algo, g["cutoff"], mp.PEEL, leaf, dA, dB, dC)
    torch.cuda.synchronize()
    return mp.to_host(dC)


def sha(C, n):
    return hashlib.sha256(np.ascontiguousarray(C[:, :n, :n]).astype("<u4").tobytes()).hexdigest()


def sampled_mismatches(C, ents, p):
    bad = []
    for i, j, s, e, mh in ents:
        want = (int(mh, 16) * (-1 if s else 1), e)
        got = I.entry(C, i, j, p)
        if got != want:
            bad.append((i, j, got, want))
    return bad


CASES = [("full_size_n1023_p256", a, a) for a in ("simple", "block", "strassen", "winograd")] + \
        [("full_size_n1024_p256", a, a) for a in ("simple", "block", "strassen", "winograd")] + \
        [("full_size_n2048_p256", a, a) for a in ("winograd", "strassen", "simple")] + \
        [("full_size_n2048_p256", "block", "simple")]


@pytest.mark.parametrize("name,algo,want_algo", CASES)
def test_whole_result_equals_oracle(name, algo, want_algo):
    g = golden(name)
    assert want_algo in g["sha256"], "golden file lacks %s" % want_algo
    C = gpu_product(g, mp.ALGOS[algo])
    got = sha(C, g["n"])
    if got != g["sha256"][want_algo]:
        bad = sampled_mismatches(C, g["entries"][want_algo], g["p"])
        pytest.fail("%s %s: whole-result digest differs from the oracle; %d of %d sampled entries differ: %s"
                    % (name, algo, len(bad), len(g["entries"][want_algo]), bad[:3]))


@pytest.mark.parametrize("algo", ["strassen", "winograd"])
def test_block_leaves_whole_result_n1024(algo):
    """The recursive products with the LDS-staged Block leaves give the same bits."""
    g = golden("full_size_n1024_p256")
    C = gpu_product(g, mp.ALGOS[algo], leaf=mp.LEAF_BLOCK)
    assert sha(C, g["n"]) == g["sha256"][algo]
