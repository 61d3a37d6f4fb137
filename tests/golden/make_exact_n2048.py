"""Write the exact reference entries of the 2048 x 2048 256-bit log-uniform
product (seeds 6 and 7) used to state the ulp error of every path.

Calls only the CPU oracle (oracle.exact: the exact dot product, then one
rounding to nearest-even at p bits) on the seeded inputs of
paper_1410_1599_amd.inputs.  The sample is a seeded 64 x 64 grid of (i, j)
plus all of row 0 and column 0.  Entries are stored as
[i, j, sign, exponent, mantissa hex] of RN_p(sum_k a_ik b_kj).  Run from the
repository root:  python tests/golden/make_exact_n2048.py  (about a minute).
"""

import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import exact, mpnum                       # noqa: E402
from paper_1410_1599_amd import inputs as I           # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def sample(n, seed=2048):
    rng = np.random.default_rng(seed)
    rows = sorted(int(v) for v in rng.choice(n, size=64, replace=False))
    cols = sorted(int(v) for v in rng.choice(n, size=64, replace=False))
    idx = {(i, j) for i in rows for j in cols}
    idx.update((0, j) for j in range(n))
    idx.update((i, 0) for i in range(n))
    return rows, cols, sorted(idx)


def main():
    n, p = 2048, 256
    A = I.log_uniform(n, n, p, 6)
    B = I.log_uniform(n, n, p, 7)
    rows, cols, idx = sample(n)
    need_r = sorted({i for i, _ in idx})
    need_c = sorted({j for _, j in idx})
    R = {i: I.row(A, i, p) for i in need_r}
    C = {j: I.col(B, j, p) for j in need_c}
    out = []
    for i, j in idx:
        nn, f = exact.exact_dot(R[i], C[j], p)
        sig, e = mpnum.rn(nn, f, p)
        out.append([i, j, 1 if sig < 0 else 0, e, "%x" % abs(sig)])
    doc = {"name": "exact_n2048_p256", "n": n, "p": p, "kind": "log_uniform", "seeds": [6, 7],
           "source": "oracle.exact: RN_p of the exact dot product", "grid_rows": rows, "grid_cols": cols,
           "entries": out}
    with open(os.path.join(HERE, "exact_n2048_p256.json"), "w") as fh:
        json.dump(doc, fh, separators=(",", ":"))
    print("wrote %d entries" % len(out))


if __name__ == "__main__":
    main()
