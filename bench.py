#!/usr/bin/env python3
"""Benchmark of the MP matrix product on one MI355X.

Workload (the metric's configuration): C := A B with m = l = n = 2048 at
256-bit precision, entries with random sign and log-uniform magnitudes over
2^-21 .. 2^20 (seeds 6 and 7), every scalar operation rounded to nearest.
One step is one full product through the C ABI with inputs resident in HBM;
the headline algorithm is Winograd's variant with cutoff 64 (odd sizes
peeled), which is bit-identical to the CPU oracle.  The other algorithms are
timed beside it.

The last line of stdout is one compact JSON object: the metric
(classical-equivalent rate 2 m l n / s), the roofline of the dominant kernel
(the grouped leaf-product launch, timed with HIP events on its own stream
during the timed steps), the CPU oracle timed on a bounded sample of the same
workload, parity of the timed result with the oracle, and short summaries of
the INT8-slice path, the LU workload, the 1023/1024 products and the serving
run.  Optional sections (the paper's grid, its LU experiment, the 8192-bit
Lotkin LU) print one JSON line each before it.
"""

import argparse
import hashlib
import json
import math
from fractions import Fraction
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# chip figures used for the roofline (256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz)
CUS, SIMDS, LANES, CLOCK_HZ = 256, 4, 16, 2.4e9
INT_LANE_OPS = CUS * SIMDS * LANES * CLOCK_HZ        # 39.3e12 32-bit VALU lane-ops/s
INT8_MFMA_PEAK_TOPS = 5000.0                         # dense INT8 MFMA, MI355X
FINAL_LINE_MAX = 4000                                # bytes of the last stdout line


def sig(x, digits=4):
    """x rounded to a few significant digits (keeps the final line short)."""
    if x is None or isinstance(x, (str, bool)) or x == 0 or not math.isfinite(x):
        return x
    return float("%.*g" % (digits, x))


def profiled_traffic(path):
    """HBM bytes per launch of the leaf kernel as measured by rocprofv3
    FETCH_SIZE / WRITE_SIZE (calibrated on a copy kernel) and recorded in a
    profile summary; None when there is none or when the kernel sources have
    changed since (the summary carries their sha256)."""
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "source_sha256"):
            k, v = line.split(":", 1)
            fields[k] = v.strip()
        if line.startswith("(sha256 over "):
            fields["files"] = line[len("(sha256 over "):].split(";")[0].rstrip(")\n").split(", ")
    if not {"traffic_bytes_per_launch", "source_sha256", "files"} <= set(fields):
        return None
    h = hashlib.sha256()
    for f in fields["files"]:
        fp = os.path.join(ROOT, f.strip())
        if not os.path.exists(fp):
            return None
        h.update(open(fp, "rb").read())
    if h.hexdigest() != fields["source_sha256"]:
        return None
    return float(fields["traffic_bytes_per_launch"])


def log10_fraction(q):
    """log10 of a positive Fraction far outside the double range."""
    def l10(v):
        sh = max(0, v.bit_length() - 64)
        return math.log10(v >> sh) + sh * math.log10(2.0)
    return l10(q.numerator) - l10(q.denominator)


def planes_sha256(C, rows, cols):
    """sha256 of the (L + 2, rows, cols) uint32 planes, little-endian, row-major."""
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(C[:, :rows, :cols]).astype("<u4").tobytes()).hexdigest()


def parse(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--prec", type=int, default=256)
    ap.add_argument("--algo", default="winograd", choices=["simple", "block", "strassen", "winograd"])
    ap.add_argument("--cutoff", type=int, default=64)
    ap.add_argument("--others", type=int, default=2, help="timed steps for each non-headline algorithm (0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0, help="target length of the CPU-oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--slice-steps", type=int, default=3, help="timed steps of the INT8-slice path (0: skip)")
    ap.add_argument("--slice-one-pass", type=int, default=0,
                    help="also time the slice product computing every diagonal in one pass (0: skip)")
    ap.add_argument("--c2", type=int, default=1,
                    help="time every algorithm on m=l=n=1023/1024 at 256 bits, uniform entries (0: skip)")
    ap.add_argument("--lu", type=int, default=1, help="run the LU workload (n=512, 512 bits, panel 64, Winograd "
                                                     "cutoff 32, random and Hilbert inputs); 0: skip")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests of the serving run (0: skip): Poisson arrivals at 0.8 x the measured "
                         "saturated rate, 90%% products / 10%% LU solves, 128/256/512 bits")
    ap.add_argument("--serve-check", type=int, default=256,
                    help="served requests recomputed alone and compared bit for bit")
    ap.add_argument("--lu-paper", type=int, default=0,
                    help="the paper's LU experiment (Section 4): no pivoting, n=1024, panel K = 32..320 with Winograd "
                         "trailing updates (cutoff 32) against column-wise LU (one panel), random at 256 bits and "
                         "Lotkin at 512 bits, x = [0..n-1]; 0: skip")
    ap.add_argument("--lotkin-8192", type=int, default=0,
                    help="the paper's 8192-bit Lotkin LU (Section 4) at this n (the paper: 1024; 0: skip): no "
                         "pivoting, Winograd trailing updates (cutoff 32) with K = 32, 64, 128 against column-wise LU, "
                         "x = [0..n-1]; times and the solution's relative error in decimal digits")
    ap.add_argument("--paper-grid", type=int, default=0,
                    help="the paper's own matrices (Section 3: a_ij = sqrt5 (i+j-1), b_ij = sqrt3 (n-i+1)), cutoff 32, "
                         "mixed odd-size policy: square n = 255..2049 and Table 5's m = n = 1024 with l = 63..513 at "
                         "128 bits, square n = 255..2048 at 1024 bits and 255..512 at 8192 bits; 0: skip")
    ap.add_argument("--launch-ab", type=int, default=0,
                    help="time the headline product under every launch shape (leaf tile width 16/32/64 columns, "
                         "a workgroup per tile or persistent grids) and the serving run with and without "
                         "persistent grids; 0: skip")
    ap.add_argument("--graph-ab", type=int, default=0,
                    help="time graph replay against eager launches for Winograd products n = 64..512 at 256 bits "
                         "(cutoff 32); 0: skip")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy a buffer of this many MiB device to device (a kernel of known traffic for "
                         "scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args(argv)


# ---------------------------------------------------------------- sections

def lu_residual_2p(mp, torch, A_host, F, piv, p):
    """||P A - L U||_inf / ||A||_inf of factors F (device, p bits) of A
    (host planes), evaluated at 2p bits on the GPU: A, L and U are widened
    exactly, P A - L U is formed by the library's Simple product and its
    subtraction at 2p bits, and the row sums of |.| by a Simple product with
    a ones column.  The evaluation's own error is below about
    n 2^(1-2p) || |L| |U| ||_inf, some 2^-p below the residual itself.
    Returns (log2 of the ratio, the ratio as a float or 0.0 below 2^-1000)."""
    import numpy as np
    n = A_host.shape[1]
    L, L2, p2 = p // 32, p // 16, 2 * p

    def widen(X):                       # (L+2, r, c) at p bits -> 2p bits, same values
        W = torch.zeros((L2 + 2,) + tuple(X.shape[1:]), dtype=torch.int32, device="cuda")
        W[L2 - L:L2] = X[:L]
        W[L2:] = X[L:]
        return W

    perm = np.arange(n)
    pv = piv.cpu().numpy()
    for k in range(n):
        r = int(pv[k])
        perm[k], perm[r] = perm[r], perm[k]
    PA = widen(mp.to_device(np.ascontiguousarray(A_host[:, perm, :])))
    F2 = widen(F)
    Lm = torch.tril(F2, diagonal=-1)
    Um = torch.triu(F2, diagonal=0)
    one = torch.zeros(L2 + 2, dtype=torch.int32, device="cuda")
    one[L2 - 1] = -2 ** 31                         # mantissa 2^(2p-1)
    one[L2] = 1                                    # exponent 1: the value 1
    idx = torch.arange(n, device="cuda")
    Lm[:, idx, idx] = one[:, None]
    LU = mp.empty(n, n, p2)
    mp.mp_gemm(n, n, n, p2, mp.SIMPLE, 0, Lm, Um, LU)
    D = mp.empty(n, n, p2)
    mp.mp_sub(n, n, p2, PA, LU, D)
    ones = one.view(L2 + 2, 1, 1).expand(L2 + 2, n, 1).contiguous()
    rows = mp.empty(n, 2, p2)

    def norm_inf(X, col):
        Y = X.clone()
        Y[L2 + 1] = 0                              # |x|
        mp.mp_gemm(n, n, 1, p2, mp.SIMPLE, 0, Y, ones, rows[:, :, col:col + 1])

    norm_inf(D, 0)
    norm_inf(PA, 1)
    torch.cuda.synchronize()
    R = mp.to_host(rows)

    def log2_entry(i, j):                          # log2 |x| from the top two limbs
        top = (int(R[L2 - 1, i, j]) << 32) | int(R[L2 - 2, i, j])
        if top == 0:
            return float("-inf")
        e = int(np.int32(np.uint32(R[L2, i, j])))
        return math.log2(top / 2.0 ** 64) + e

    lr = max(log2_entry(i, 0) for i in range(n))
    la = max(log2_entry(i, 1) for i in range(n))
    l2 = lr - la
    return l2, (2.0 ** l2 if l2 > -1000 else 0.0)


def headline(args, mp, torch, I, A, B):
    n, p = args.n, args.prec
    L = p // 32
    dA, dB = mp.to_device(A), mp.to_device(B)
    dC = mp.empty(n, n, p)
    algo = mp.ALGOS[args.algo]

    def step(al=algo):
        mp.mp_gemm_ex(n, n, n, p, al, args.cutoff, mp.PEEL, mp.LEAF_SIMPLE, dA, dB, dC)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    mp.mp_profile_read()                     # drop anything recorded before
    mp.mp_profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mp.mp_profile(False)
    recs = mp.mp_profile_read()
    ms = (t1 - t0) * 1e3 / args.steps

    # dominant kernel: the grouped leaf-product launch
    leaf = [r for r in recs if r["kind"] == 0]
    leaf_ms = sum(r["ms"] for r in leaf) / max(1, len(leaf))
    leaf_units = leaf[0]["units"] if leaf else 0.0          # scalar MP multiply-adds per launch
    all_ms = sum(r["ms"] for r in recs) / max(1, args.steps)
    achieved = leaf_units * L * L / (leaf_ms * 1e-3) / 1e12 if leaf_ms > 0 else 0.0
    peak = INT_LANE_OPS / 1e12
    roofline = {
        "bound": "alu", "achieved": sig(achieved), "peak": sig(peak), "unit": "TOP/s",
        "frac": sig(achieved / peak),
        "traffic": profiled_traffic(os.path.join(ROOT, "profiles", "leaf_gemm_simple_L%d_n%d_p%d_%s.md"
                                                 % (L, n, p, args.algo))) if args.cutoff == 64 else None,
        "kernel": "k_gemm_simple<L=%d> grouped leaf products" % L,
        "op": "32x32->64-bit limb multiply-accumulate, L^2=%d per MP multiply-add" % (L * L),
        "launch_ms": sig(leaf_ms), "units_per_launch": leaf_units,
        "leaf_share_of_step": sig(leaf_ms / all_ms) if all_ms else None,
    }
    C = mp.to_host(dC)

    # parity of the timed result: the sha256 of the whole result against the
    # C oracle's (stored by tests/golden/make_full_size.py), else its samples
    parity = None
    gold = os.path.join(ROOT, "tests", "golden", "full_size_n%d_p%d.json" % (n, p))
    if os.path.exists(gold) and args.cutoff == 64:
        g = json.load(open(gold))
        if g["kind"] == "log_uniform" and list(g["seeds"]) == [6, 7]:
            want = g.get("sha256", {}).get(args.algo)
            if want:
                ok = planes_sha256(C, n, n) == want
                parity = ("whole %dx%d result bit-identical to the C oracle (sha256)" % (n, n) if ok
                          else "MISMATCH: the %dx%d result differs from the C oracle (sha256)" % (n, n))
            elif args.algo in g.get("entries", {}):
                ents = g["entries"][args.algo]
                bad = sum(1 for i, j, s, e, mh in ents
                          if I.entry(C, i, j, p) != (int(mh, 16) * (-1 if s else 1), e))
                parity = "%d of %d sampled entries bit-exact vs the oracle" % (len(ents) - bad, len(ents))

    others = {}
    if args.others > 0:
        for name in ("simple", "block", "strassen", "winograd"):
            if name == args.algo:
                continue
            al = mp.ALGOS[name]
            step(al)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.others):
                step(al)
            torch.cuda.synchronize()
            others[name] = sig((time.perf_counter() - t0) / args.others * 1e3)
    return {"ms": ms, "rate": 2.0 * n ** 3 / (ms * 1e-3), "roofline": roofline, "C": C, "parity": parity,
            "others_ms": others, "dA": dA, "dB": dB, "dC": dC}


def slice_section(args, mp, torch, h):
    n, p = args.n, args.prec
    dA, dB = h["dA"], h["dB"]
    dS = mp.empty(n, n, p)
    mp.mp_gemm_slice(n, n, n, p, 64, dA, dB, dS)
    torch.cuda.synchronize()
    mp.mp_profile_read()
    mp.mp_profile(True)
    t0 = time.perf_counter()
    for _ in range(args.slice_steps):
        win = mp.mp_gemm_slice(n, n, n, p, 64, dA, dB, dS)
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / args.slice_steps
    mp.mp_profile(False)
    srecs = mp.mp_profile_read()
    # first pass of the early stop (diagonals u >= u0, every tile): the
    # dominant launch; the second pass runs only for undecided tiles
    mm = [r for r in srecs if r["kind"] == 2 and r["op"] == 0]
    mm2 = [r for r in srecs if r["kind"] == 2 and r["op"] == 1]
    mm_ms = sum(r["ms"] for r in mm) / max(1, len(mm))
    mm_tops = mm[0]["units"] / (mm_ms * 1e-3) / 1e12 if mm else 0.0
    u0, ndiag, recomputed, ntiles, _ = mp.mp_slice_last()
    out = {
        "value": sig(2.0 * n ** 3 / ts), "ms_per_step": sig(ts * 1e3), "speedup_vs_limb": sig(h["ms"] / (ts * 1e3)),
        "windows": list(win),
        "roofline": {"bound": "mfma", "achieved": sig(mm_tops), "peak": INT8_MFMA_PEAK_TOPS, "unit": "TOP/s int8",
                     "frac": sig(mm_tops / INT8_MFMA_PEAK_TOPS), "kernel": "k_slice_gemm v_mfma_i32_32x32x32_i8",
                     "launch_ms": sig(mm_ms)},
        "other_ms": sig(sum(r["ms"] for r in srecs if r["kind"] == 3) / args.slice_steps),
        "early_stop": {"u0": u0, "diagonals": ndiag, "tiles_recomputed": recomputed, "tiles": ntiles,
                       "second_pass_ms": sig(sum(r["ms"] for r in mm2) / args.slice_steps)},
    }
    if args.slice_one_pass:
        mp.mp_set_slice_guard(-1)
        mp.mp_gemm_slice(n, n, n, p, 64, dA, dB, dS)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.slice_steps):
            mp.mp_gemm_slice(n, n, n, p, 64, dA, dB, dS)
        torch.cuda.synchronize()
        out["early_stop"]["one_pass_ms_per_step"] = sig((time.perf_counter() - t1) / args.slice_steps * 1e3)
        mp.mp_set_slice_guard(32)
        mp.mp_gemm_slice(n, n, n, p, 64, dA, dB, dS)
    S = mp.to_host(dS)
    del dS
    return out, S


def accuracy_section(args, I, results):
    """Max ulp error against stored exact products (RN_p of the exact dot
    product, written by tests/golden/make_exact_n2048.py)."""
    n, p = args.n, args.prec
    gold = os.path.join(ROOT, "tests", "golden", "exact_n%d_p%d.json" % (n, p))
    if not os.path.exists(gold):
        return None
    g = json.load(open(gold))
    if g["kind"] != "log_uniform" or list(g["seeds"]) != [6, 7]:
        return None

    def ulps(x, c):
        (sx, ex), (sc, ec) = x, c
        if sc == 0:
            return 0.0 if sx == 0 else float("inf")
        return float(abs(Fraction(sx) * Fraction(2) ** (ex - ec) - sc))

    res = {}
    for name, host in results.items():
        if host is None:
            continue
        worst = 0.0
        for i, j, s, e, mh in g["entries"]:
            worst = max(worst, ulps(I.entry(host, i, j, p), (int(mh, 16) * (-1 if s else 1), e)))
        res[name] = sig(worst)
    res["entries"] = len(g["entries"])
    return res


def lu_section(mp, torch, I):
    """The LU workload: n = 512, 512 bits, panel 64, Winograd trailing updates
    with cutoff 32; random and Hilbert inputs, b = A * ones."""
    out = {}
    pl, nl = 512, 512
    for kind in ("random", "hilbert"):
        Ah = I.uniform_pm1(nl, nl, pl, 5) if kind == "random" else I.hilbert(nl, pl)
        ones = mp.to_device(I.ones_column(nl, pl))
        dAl = mp.to_device(Ah)
        dx = mp.empty(nl, 1, pl)
        piv = torch.zeros(nl, dtype=torch.int32, device="cuda")
        mp.mp_gemm(nl, nl, 1, pl, mp.SIMPLE, 0, dAl, ones, dx)          # b = A * ones
        work = dAl.clone()
        mp.mp_lu_ex(nl, pl, work, piv, 64, mp.WINOGRAD, 32)              # warm plans
        tl, tsv = [], []
        for _ in range(3):
            work.copy_(dAl)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            info = mp.mp_lu_ex(nl, pl, work, piv, 64, mp.WINOGRAD, 32)
            torch.cuda.synchronize()
            tl.append(time.perf_counter() - t0)
            dxx = dx.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            mp.mp_lu_solve(nl, pl, work, piv, dxx)
            torch.cuda.synchronize()
            tsv.append(time.perf_counter() - t0)
        t_lu, t_solve = min(tl), min(tsv)
        xh = mp.to_host(dxx)
        err = max(abs(Fraction(s) * Fraction(2) ** (e - pl) - 1)
                  for s, e in (I.entry(xh, i, 0, pl) for i in range(nl)))
        l2, _ = lu_residual_2p(mp, torch, Ah, work, piv, pl)
        out[kind] = {"info": info, "lu_ms": sig(t_lu * 1e3), "solve_ms": sig(t_solve * 1e3),
                     "rate": sig((2.0 * nl ** 3 / 3) / t_lu), "residual_log2": round(l2, 2),
                     "max_abs_x_minus_1_log10": round(log10_fraction(err), 2) if err else None}
    return out


def c2_section(mp, torch, I):
    """m = l = n = 1023 and 1024 at 256 bits, uniform entries (seeds 3/4):
    every algorithm at cutoff 64 with odd sizes peeled (parity: a GPU test)."""
    out = {}
    for nn in (1023, 1024):
        dA2 = mp.to_device(I.uniform_pm1(nn, nn, 256, 3))
        dB2 = mp.to_device(I.uniform_pm1(nn, nn, 256, 4))
        dC2 = mp.empty(nn, nn, 256)
        out[nn] = {}
        for name in ("simple", "block", "strassen", "winograd"):
            best = float("inf")
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                mp.mp_gemm_ex(nn, nn, nn, 256, mp.ALGOS[name], 64, mp.PEEL, mp.LEAF_SIMPLE, dA2, dB2, dC2)
                torch.cuda.synchronize()
                best = min(best, time.perf_counter() - t0)
            out[nn][name] = sig(best * 1e3)
        del dA2, dB2, dC2
    return out


def serve_section(args, mp, torch):
    import numpy as np
    from paper_1410_1599_amd import serve
    torch.cuda.empty_cache()
    srv = serve.Server(slots=4)
    sat = serve.saturated_rate(srv)
    reqs = serve.make_requests(args.serve_requests, 0.8 * sat, seed=8)
    rng = np.random.default_rng(3)
    chk = set(int(v) for v in rng.choice(len(reqs), size=min(args.serve_check, len(reqs)), replace=False))
    srv.keep = chk
    st = srv.run(reqs)
    ref = srv.alone([r for r in reqs if r.rid in chk])
    same = sum(1 for r in reqs if r.rid in chk and r.result is not None and np.array_equal(ref[r.rid], r.result))
    return {"requests": st["requests"], "p50_ms": sig(st["p50_ms"]), "p99_ms": sig(st["p99_ms"]),
            "req_per_s": sig(st["req_per_s"]), "gemm_2mln_per_s": sig(st["gemm_2mln_per_s"]),
            "saturated_req_per_s": sig(sat), "arrival_rate": sig(0.8 * sat),
            "peak_admitted_gb": sig(st["peak_admitted_gb"]), "failed": st.get("failed", 0),
            "identical_alone_vs_mix": "%d/%d" % (same, len(chk))}


def cpu_baseline(args, A, B):
    """The C oracle (oracle/c/mpref.c, untuned, all host threads) running the
    headline algorithm on the leading ns x ns blocks of the same inputs, ns
    sized by a short probe so the sample takes about --cpu-seconds."""
    import numpy as np
    from oracle import cref
    n, p = args.n, args.prec
    cores = cref.threads()

    def run(ns):
        a = np.ascontiguousarray(A[:, :ns, :ns])
        b = np.ascontiguousarray(B[:, :ns, :ns])
        t0 = time.perf_counter()
        cref.gemm(a, b, p, algo=args.algo, cutoff=args.cutoff, policy="peel")
        return time.perf_counter() - t0

    probe = min(256, n)
    tp = run(probe)
    # classical work scales as ns^3; the recursion saves a little more
    ns = int(probe * (args.cpu_seconds / max(tp, 1e-3)) ** (1.0 / 3.0)) // 64 * 64
    ns = max(probe, min(n, ns))
    t = run(ns)
    return {"value": sig(2.0 * ns ** 3 / t), "unit": "2mln/s", "cores": cores, "kind": "oracle",
            "sample": "C oracle %s (cutoff %d, peel) on the leading %dx%d blocks of the same %d-bit log-uniform "
                      "A and B, %.1f s on %d threads" % (args.algo, args.cutoff, ns, ns, p, t, cores)}


def final_line(args, h, cpu=None, slice_res=None, accuracy=None, lu=None, c2=None, serve_res=None):
    """The compact summary printed as the last stdout line."""
    n, p = args.n, args.prec
    out = {
        "metric": "MP-GEMM 2mln/s at 256-bit n=2048 (limb path; INT8-slice path and serve p50/p99 ms beside it)",
        "value": sig(h["rate"], 6), "unit": "2mln/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sig(h["ms"], 6), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "mp_gemm m=l=n=%d prec=%d %s cutoff=%d peel, log-uniform |a| in 2^-21..2^20, "
                               "seeds 6/7" % (n, p, args.algo, args.cutoff),
                   "m": n, "l": n, "n": n, "prec": p, "algo": args.algo, "cutoff": args.cutoff},
        "roofline": h["roofline"], "cpu_baseline": cpu, "parity": h["parity"], "others_ms": h["others_ms"],
        "slice": slice_res, "max_ulp_vs_exact": accuracy, "lu_n512_p512": lu, "c2_ms": c2, "serve": serve_res,
    }
    return out


def launch_ab_section(args, mp, torch, h):
    """ms per step of the headline product for every launch shape."""
    n, p = args.n, args.prec
    out = {"section": "launch_ab", "config": "mp_gemm m=l=n=%d prec=%d %s cutoff=%d; min over 3 runs of %d steps"
                                             % (n, p, args.algo, args.cutoff, max(2, args.steps // 4))}
    for tcl in (0, 5, 4):
        for persist in (0, 1):
            mp.mp_set_launch(tcl, persist)
            try:
                mp.mp_gemm(n, n, n, p, mp.ALGOS[args.algo], args.cutoff, h["dA"], h["dB"], h["dC"])
                best = float("inf")
                for _ in range(3):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(max(2, args.steps // 4)):
                        mp.mp_gemm(n, n, n, p, mp.ALGOS[args.algo], args.cutoff, h["dA"], h["dB"], h["dC"])
                    torch.cuda.synchronize()
                    best = min(best, (time.perf_counter() - t0) / max(2, args.steps // 4))
            finally:
                mp.mp_set_launch(0, 0)
            out["tile_cols_%d_%s" % (64 if tcl == 0 else 1 << tcl, "persistent" if persist else "per_tile")] = \
                sig(best * 1e3)
    return out


def graph_ab_section(mp, torch, I):
    """Eager launches against graph replay for small products (launch-bound)."""
    p = 256
    out = {"section": "graph_ab", "config": "mp_gemm n x n x n, 256 bits, Winograd cutoff 32, on a side stream; "
                                            "ms per product, mean of 50 after one warm call"}
    s = torch.cuda.Stream()
    for n in (64, 128, 256, 512):
        A = mp.to_device(I.uniform_pm1(n, n, p, 71))
        B = mp.to_device(I.uniform_pm1(n, n, p, 72))
        C = mp.empty(n, n, p)
        info = mp.mp_plan_info(n, n, n, p, mp.WINOGRAD, 32)
        row = {"launches": info["n_launches"]}
        with torch.cuda.stream(s):
            for mode in (0, 1):
                mp.mp_set_graph_mode(mode)
                try:
                    s.synchronize()
                    t0 = time.perf_counter()
                    mp.mp_gemm(n, n, n, p, mp.WINOGRAD, 32, A, B, C)      # plan (and capture) on first use
                    s.synchronize()
                    first = time.perf_counter() - t0
                    t0 = time.perf_counter()
                    for _ in range(50):
                        mp.mp_gemm(n, n, n, p, mp.WINOGRAD, 32, A, B, C)
                    s.synchronize()
                    row["graph" if mode else "eager"] = sig((time.perf_counter() - t0) / 50 * 1e3)
                    if mode:
                        row["capture_ms"] = sig(first * 1e3)
                finally:
                    mp.mp_set_graph_mode(0)
        out[n] = row
    return out


def extended_sections(args, mp, torch, I):
    """Opt-in sections, each printed as its own JSON line."""
    if args.lu_paper:
        res = {"section": "lu_paper", "config": "n=1024, no pivoting, Winograd trailing updates with cutoff 32; "
                                                 "b = A x with x = [0..n-1] by Simple; second of two runs per K"}
        npl = 1024
        for kind, pl in (("random", 256), ("lotkin", 512)):
            Ah = I.uniform_pm1(npl, npl, pl, 5) if kind == "random" else I.lotkin(npl, pl)
            dAl = mp.to_device(Ah)
            xt = mp.to_device(I.arange_column(npl, pl))
            db = mp.empty(npl, 1, pl)
            mp.mp_gemm(npl, npl, 1, pl, mp.SIMPLE, 0, dAl, xt, db)
            work = dAl.clone()
            piv = torch.zeros(npl, dtype=torch.int32, device="cuda")
            times = {}
            for K in [32 * a for a in range(1, 11)] + [npl]:
                for _ in range(2):
                    work.copy_(dAl)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    mp.mp_lu_nopivot(npl, pl, work, piv, K, mp.WINOGRAD, 32)
                    torch.cuda.synchronize()
                    tk = time.perf_counter() - t0
                times["column-wise" if K == npl else "K=%d" % K] = round(tk * 1e3, 2)
            bestK = min((k for k in times if k != "column-wise"), key=lambda k: times[k])
            work.copy_(dAl)
            info = mp.mp_lu_nopivot(npl, pl, work, piv, int(bestK[2:]), mp.WINOGRAD, 32)
            dx = db.clone()
            mp.mp_lu_solve(npl, pl, work, piv, dx)
            xh = mp.to_host(dx)
            err = max(abs(Fraction(s) * Fraction(2) ** (e - pl) - i)
                      for i, (s, e) in enumerate(I.entry(xh, i, 0, pl) for i in range(npl)))
            res[kind] = {"prec": pl, "info": info, "lu_ms": times, "best": bestK,
                         "time_saved_vs_columnwise": round(1 - times[bestK] / times["column-wise"], 4),
                         "max_abs_x_minus_xtrue": float(err)}
            del dAl, work, db, dx
        print(json.dumps(res), flush=True)

    if args.lotkin_8192:
        pw, nw = 8192, args.lotkin_8192
        dAw = mp.to_device(I.lotkin(nw, pw))
        dbw = mp.empty(nw, 1, pw)
        mp.mp_gemm(nw, nw, 1, pw, mp.SIMPLE, 0, dAw, mp.to_device(I.arange_column(nw, pw)), dbw)
        work = dAw.clone()
        piv = torch.zeros(nw, dtype=torch.int32, device="cuda")
        times, digits = {}, {}
        for K in (32, 64, 128, nw):
            for _ in range(2):
                work.copy_(dAw)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = mp.mp_lu_nopivot(nw, pw, work, piv, K, mp.WINOGRAD, 32)
                torch.cuda.synchronize()
                tk = time.perf_counter() - t0
            name = "column-wise" if K == nw else "K=%d" % K
            times[name] = round(tk * 1e3, 1)
            dx = dbw.clone()
            mp.mp_lu_solve(nw, pw, work, piv, dx)
            xh = mp.to_host(dx)
            worst = max(abs(Fraction(s) * Fraction(2) ** (e - pw) - i) / i
                        for i, (s, e) in ((i, I.entry(xh, i, 0, pw)) for i in range(1, nw)))
            digits[name] = round(-log10_fraction(worst), 1) if worst > 0 else None
        # the paper's remedy: Winograd's updates at more bits (it used 8650; the
        # next width here is 10240) against column-wise LU at 8192 bits
        more = {}
        pm = 10240
        Am = mp.to_device(I.lotkin(nw, pm))
        dbm = mp.empty(nw, 1, pm)
        mp.mp_gemm(nw, nw, 1, pm, mp.SIMPLE, 0, Am, mp.to_device(I.arange_column(nw, pm)), dbm)
        wm = Am.clone()
        for K in (64, 128):
            for _ in range(2):
                wm.copy_(Am)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                mp.mp_lu_nopivot(nw, pm, wm, piv, K, mp.WINOGRAD, 32)
                torch.cuda.synchronize()
                tk = time.perf_counter() - t0
            dx = dbm.clone()
            mp.mp_lu_solve(nw, pm, wm, piv, dx)
            xh = mp.to_host(dx)
            worst = max(abs(Fraction(s) * Fraction(2) ** (e - pm) - i) / i
                        for i, (s, e) in ((i, I.entry(xh, i, 0, pm)) for i in range(1, nw)))
            more["K=%d" % K] = {"lu_ms": round(tk * 1e3, 1),
                                "correct_decimal_digits_of_x": round(-log10_fraction(worst), 1),
                                "time_saved_vs_columnwise_8192": round(1 - tk * 1e3 / times["column-wise"], 4)}
        del Am, wm, dbm
        bestK = min((k for k in times if k != "column-wise"), key=lambda k: times[k])
        print(json.dumps({"section": "lotkin_8192", "n": nw, "prec": pw, "info": info, "lu_ms": times,
                          "best": bestK, "winograd_at_10240_bits": more,
                          "time_saved_vs_columnwise": round(1 - times[bestK] / times["column-wise"], 4),
                          "correct_decimal_digits_of_x": digits,
                          "config": "Lotkin matrix, no pivoting, Winograd trailing updates with cutoff 32, b = A x "
                                    "with x = [0..n-1] by Simple at 8192 bits; second of two runs"}), flush=True)
        del dAw, work, dbw

    if args.paper_grid:
        from math import isqrt

        def rel_err(C, m, l, n, pg):
            # rows 0, m/2, m-1, every column; exact c_ij = sqrt15 R_i to 3p fraction bits
            tail = sum(k * (n - k + 1) for k in range(1, l + 1))
            worst = Fraction(0)
            for i in sorted({0, m // 2, m - 1}):
                R = i * l * (2 * n - l + 1) // 2 + tail
                K = 3 * pg
                X = Fraction(isqrt(15 * R * R << (2 * K)), 1 << K)
                for j in range(n):
                    s, e = I.entry(C, i, j, pg)
                    worst = max(worst, abs(Fraction(s) * Fraction(2) ** (e - pg) - X) / X)
            return worst

        def run(m, l, n, algos, pg=128):
            A8, B8 = I.sqrt_workload(m, l, n, pg)
            dA8, dB8, dC8 = mp.to_device(A8), mp.to_device(B8), mp.empty(m, n, pg)
            out = {}
            for name in algos:
                al = mp.ALGOS[name]
                for _ in range(2):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    mp.mp_gemm_ex(m, l, n, pg, al, 32, mp.MIXED, mp.LEAF_SIMPLE, dA8, dB8, dC8)
                    torch.cuda.synchronize()
                    tk = time.perf_counter() - t0
                worst = rel_err(mp.to_host(dC8), m, l, n, pg)
                out[name] = {"ms": round(tk * 1e3, 3), "2mln_per_s": sig(2.0 * m * l * n / tk),
                             "max_rel_err_sampled_log10": round(log10_fraction(worst), 2) if worst else None}
            return out

        grid = {"section": "paper_grid", "config": "cutoff 32, mixed policy; relative errors on rows 0, m/2, m-1",
                "square": {}, "table5_m_n_1024": {}, "square_1024bit": {}, "square_8192bit": {}}
        for nn in (255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 2047, 2048, 2049):
            grid["square"][nn] = run(nn, nn, nn, ("simple", "block", "strassen", "winograd"))
        for ll in (63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513):
            grid["table5_m_n_1024"][ll] = run(1024, ll, 1024, ("simple", "strassen", "winograd"))
        for nn in (255, 256, 511, 512, 1023, 1024, 2048):
            grid["square_1024bit"][nn] = run(nn, nn, nn, ("simple", "block", "strassen", "winograd")
                                             if nn <= 1024 else ("strassen", "winograd"), pg=1024)
        for nn in (255, 256, 511, 512):
            grid["square_8192bit"][nn] = run(nn, nn, nn, ("simple", "block", "strassen", "winograd")
                                             if nn <= 256 else ("strassen", "winograd"), pg=8192)
        print(json.dumps(grid), flush=True)


def main(argv=None):
    args = parse(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (--gpus %d refused)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1410_1599_amd import inputs as I
    from paper_1410_1599_amd import mp

    if args.copy_probe_mib:
        src = torch.empty(args.copy_probe_mib << 18, dtype=torch.int32, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)          # reads and writes copy_probe_mib MiB each, kernel named "neg"
        torch.cuda.synchronize()
        del src, dst

    n, p = args.n, args.prec
    A = I.log_uniform(n, n, p, 6)
    B = I.log_uniform(n, n, p, 7)
    h = headline(args, mp, torch, I, A, B)
    print("# headline %.3f ms/step, parity: %s" % (h["ms"], h["parity"]), file=sys.stderr, flush=True)

    if args.launch_ab:
        print(json.dumps(launch_ab_section(args, mp, torch, h)), flush=True)
    if args.graph_ab:
        print(json.dumps(graph_ab_section(mp, torch, I)), flush=True)

    slice_res, slice_host = None, None
    if args.slice_steps > 0:
        slice_res, slice_host = slice_section(args, mp, torch, h)
    accuracy = accuracy_section(args, I, {"limb_" + args.algo: h["C"], "slice": slice_host})
    del h["dA"], h["dB"], h["dC"]
    torch.cuda.empty_cache()
    lu = lu_section(mp, torch, I) if args.lu else None
    c2 = c2_section(mp, torch, I) if args.c2 else None
    serve_res = serve_section(args, mp, torch) if args.serve_requests > 0 else None
    if args.launch_ab and args.serve_requests > 0:
        mp.mp_set_launch(0, 1)
        try:
            alt = serve_section(args, mp, torch)
        finally:
            mp.mp_set_launch(0, 0)
        print(json.dumps({"section": "serve_launch_ab", "per_tile": serve_res, "persistent": alt}), flush=True)
    extended_sections(args, mp, torch, I)
    cpu = None if args.no_cpu else cpu_baseline(args, A, B)

    line = json.dumps(final_line(args, h, cpu, slice_res, accuracy, lu, c2, serve_res), separators=(",", ":"))
    if len(line) > FINAL_LINE_MAX:
        print("# warning: final line is %d bytes" % len(line), file=sys.stderr)
    print(line, flush=True)


if __name__ == "__main__":
    main()
