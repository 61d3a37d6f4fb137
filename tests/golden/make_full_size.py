"""Write the full-size expected products used by the GPU parity tests.

Calls only the CPU oracle (oracle.cref, the C twin of oracle/gemm.py) on the
seeded synthetic inputs of paper_1410_1599_amd.inputs, computes each full
product once, and stores the sha256 of the whole result (its L + 2 planes as
little-endian uint32, row-major, ld = n) and a fixed sample of its entries
(for the message when a digest differs):

* full_size_n1023_p256.json, full_size_n1024_p256.json: 256-bit products of
  uniform (-1, 1) matrices (seeds 3 and 4): Simple, Block (block 16),
  Strassen and Winograd with cutoff 64 and odd sizes peeled;
* full_size_n2048_p256.json: 2048 x 2048 at 256 bits, entries with
  log-uniform magnitudes over 2^-21 .. 2^20 (seeds 6 and 7): Winograd,
  Strassen and Simple with cutoff 64 (Block equals Simple bit for bit, an
  oracle invariant pinned on the CPU).

Entries are stored as [i, j, sign, exponent, mantissa hex].  Run from the
repository root:  python tests/golden/make_full_size.py [name ...]  (about an
hour on eight cores for all three files).
"""

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import cref                               # noqa: E402
from paper_1410_1599_amd import inputs as I           # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

CONFIGS = [
    dict(name="full_size_n1023_p256", n=1023, p=256, kind="uniform", seeds=(3, 4),
         algos=("winograd", "strassen", "simple", "block"), cutoff=64, policy="peel"),
    dict(name="full_size_n1024_p256", n=1024, p=256, kind="uniform", seeds=(3, 4),
         algos=("winograd", "strassen", "simple", "block"), cutoff=64, policy="peel"),
    dict(name="full_size_n2048_p256", n=2048, p=256, kind="log_uniform", seeds=(6, 7),
         algos=("winograd", "strassen", "simple"), cutoff=64, policy="peel"),
]


def make_inputs(cfg):
    n, p = cfg["n"], cfg["p"]
    gen = I.uniform_pm1 if cfg["kind"] == "uniform" else I.log_uniform
    return gen(n, n, p, cfg["seeds"][0]), gen(n, n, p, cfg["seeds"][1])


def sample_indices(n, seed=12345):
    """First and last row and column at stride 7, the four corners, and 512
    seeded random positions."""
    rng = np.random.default_rng(seed)
    idx = set()
    for t in range(0, n, 7):
        idx.update({(0, t), (n - 1, t), (t, 0), (t, n - 1)})
    idx.update({(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1)})
    for i, j in rng.integers(0, n, size=(512, 2)):
        idx.add((int(i), int(j)))
    return sorted(idx)


def planes_sha256(C, n):
    return hashlib.sha256(np.ascontiguousarray(C[:, :n, :n]).astype("<u4").tobytes()).hexdigest()


def main(only=None):
    for cfg in CONFIGS:
        if only and cfg["name"] not in only:
            continue
        A, B = make_inputs(cfg)
        idx = sample_indices(cfg["n"])
        out = {k: v for k, v in cfg.items() if k != "algos"}
        out["source"] = "oracle.cref.gemm (C oracle): sha256 of the whole result, and sampled entries"
        out["entries"] = {}
        out["sha256"] = {}
        for algo in cfg["algos"]:
            t = time.time()
            C = cref.gemm(A, B, cfg["p"], algo=algo, cutoff=cfg["cutoff"], policy=cfg["policy"])
            ents = []
            for i, j in idx:
                sig, e = I.entry(C, i, j, cfg["p"])
                ents.append([i, j, 1 if sig < 0 else 0, e, "%x" % abs(sig)])
            out["entries"][algo] = ents
            out["sha256"][algo] = planes_sha256(C, cfg["n"])
            print(cfg["name"], algo, "%.1fs" % (time.time() - t), flush=True)
        with open(os.path.join(HERE, cfg["name"] + ".json"), "w") as f:
            json.dump(out, f, separators=(",", ":"))


if __name__ == "__main__":
    main(sys.argv[1:] or None)
