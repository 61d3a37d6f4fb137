"""Write the expected results of the wide-precision GPU parity tests
(2048, 4096, 8192 and 10240 bits) at sizes that span several 256-element tiles of
the one-value-per-wavefront kernels and two or more recursion levels.

Calls only the CPU oracle (oracle.cref, the wide build of the C twin of
oracle/gemm.py and oracle/lu.py, pinned to the Python oracle at these
precisions by tests/test_oracle_wide_twin.py) on the seeded synthetic inputs
of paper_1410_1599_amd.inputs.  For each case it stores the sha256 of the
whole result (planes as little-endian uint32, row-major, ld = the column
count) and a fixed sample of entries for the message when a digest differs.
LU cases also store the pivots and info, and the solution of A x = b.

    python tests/golden/make_wide.py [case ...]     (a few minutes on 8 cores)
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
OUT = os.path.join(HERE, "wide_parity.json")

# (name, p, m, l, n, algo, cutoff, policy, input seeds)
GEMMS = [
    ("p2048_n128_winograd", 2048, 128, 128, 128, "winograd", 32, "peel", (11, 12)),
    ("p2048_n128_strassen", 2048, 128, 128, 128, "strassen", 32, "peel", (11, 12)),
    ("p2048_n128_simple", 2048, 128, 128, 128, "simple", 0, "peel", (11, 12)),
    ("p2048_ragged_winograd", 2048, 97, 130, 75, "winograd", 16, "peel", (13, 14)),
    ("p8192_n64_winograd", 8192, 64, 64, 64, "winograd", 16, "peel", (15, 16)),
    ("p8192_n64_strassen", 8192, 64, 64, 64, "strassen", 16, "peel", (15, 16)),
    ("p8192_ragged_winograd_mixed", 8192, 65, 70, 66, "winograd", 16, "mixed", (17, 18)),
    ("p8192_n128_winograd", 8192, 128, 128, 128, "winograd", 32, "peel", (25, 26)),
    ("p4096_n96_strassen", 4096, 96, 96, 96, "strassen", 16, "peel", (27, 28)),
    ("p10240_n64_winograd", 10240, 64, 64, 64, "winograd", 16, "peel", (19, 20)),
    ("p10240_ragged_strassen_pad", 10240, 61, 67, 70, "strassen", 15, "pad", (21, 22)),
]

# (name, p, n, kind, pivot, panel, algo, cutoff)
LUS = [
    ("lu_p8192_n64_random", 8192, 64, "random", True, 16, "winograd", 8),
    ("lu_p8192_n64_lotkin_nopivot", 8192, 64, "lotkin", False, 16, "winograd", 8),
    ("lu_p2048_n96_hilbert", 2048, 96, "hilbert", True, 32, "winograd", 16),
]


def sha(C, rows, cols):
    return hashlib.sha256(np.ascontiguousarray(C[:, :rows, :cols]).astype("<u4").tobytes()).hexdigest()


def samples(C, rows, cols, p, count=64, seed=5):
    rng = np.random.default_rng(seed)
    idx = {(0, 0), (rows - 1, cols - 1), (0, cols - 1), (rows - 1, 0)}
    idx.update((int(i), int(j)) for i, j in zip(rng.integers(0, rows, count), rng.integers(0, cols, count)))
    out = []
    for i, j in sorted(idx):
        s, e = I.entry(C, i, j, p)
        out.append([i, j, 1 if s < 0 else 0, e, "%x" % abs(s)])
    return out


def lu_input(kind, n, p):
    if kind == "random":
        return I.uniform_pm1(n, n, p, 23)
    if kind == "hilbert":
        return I.hilbert(n, p)
    return I.lotkin(n, p)


def rhs(A, kind, n, p):
    """b = A x by the oracle's Simple product: x = ones, or [0..n-1] for the
    unpivoted Lotkin case (the paper's experiment)."""
    x = I.arange_column(n, p) if kind == "lotkin" else I.ones_column(n, p)
    return cref.gemm(A, x, p, algo="simple")


def main(only=None):
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name, p, m, l, n, algo, cut, policy, seeds in GEMMS:
        if only and name not in only:
            continue
        t = time.time()
        A = I.uniform_pm1(m, l, p, seeds[0])
        B = I.uniform_pm1(l, n, p, seeds[1])
        C = cref.gemm(A, B, p, algo=algo, cutoff=max(cut, 1), policy=policy)
        res[name] = {"kind": "gemm", "p": p, "m": m, "l": l, "n": n, "algo": algo, "cutoff": cut, "policy": policy,
                     "seeds": list(seeds), "inputs": "uniform_pm1", "sha256": sha(C, m, n),
                     "entries": samples(C, m, n, p)}
        print(name, "%.1fs" % (time.time() - t), flush=True)
        json.dump(res, open(OUT, "w"), separators=(",", ":"), sort_keys=True)
    for name, p, n, kind, pivot, panel, algo, cut in LUS:
        if only and name not in only:
            continue
        t = time.time()
        A = lu_input(kind, n, p)
        b = rhs(A, kind, n, p)
        F, piv, info = cref.lu(A, p, panel=panel, algo=algo, cutoff=cut, pivot=pivot)
        x = cref.lu_solve(F, piv, b, p)
        res[name] = {"kind": "lu", "p": p, "n": n, "input": kind, "pivot": pivot, "panel": panel, "algo": algo,
                     "cutoff": cut, "info": info, "piv": [int(v) for v in piv], "sha256": sha(F, n, n),
                     "b_sha256": sha(b, n, 1), "x_sha256": sha(x, n, 1), "entries": samples(F, n, n, p)}
        print(name, "%.1fs" % (time.time() - t), flush=True)
        json.dump(res, open(OUT, "w"), separators=(",", ":"), sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or None)
