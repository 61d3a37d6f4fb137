"""Request loop for MP GEMMs and LU solves of mixed sizes and precisions.

Continuous batching on one GPU:

* requests arrive by a seeded Poisson process; a request is a product
  C = AB (m, l, n each log-uniform in [32, 1024]) or a linear solve
  (n log-uniform in [64, 512]: b = A 1, LU with partial pivoting, solve),
  at 128, 256 or 512 bits, with operands uniform on (-1, 1);
* the loop keeps `slots` HIP streams; whenever a slot is free it admits the
  waiting requests in arrival order while their HBM footprint (operands,
  result and the library's workspace for that shape) fits the budget:
  products of the head request's precision are grouped into one batched call
  (every recursion level of every product in one grouped launch, all leaves
  in one), a solve runs alone; work on different slots overlaps on the
  device, and a request that arrives meanwhile joins the next free slot;
* operands are generated on the device from the request's seed and never
  leave it; completion is a GPU event, and latency is measured from the
  arrival time to that event on the GPU clock.

`run()` returns p50 / p99 latency, throughput and the classical-equivalent
rate of the products.  The results of a sampled subset are kept so that
`alone()` can recompute them one at a time and compare them bit for bit.
"""

import argparse
import json
import math
import time

import numpy as np

from . import mp


class Request:
    __slots__ = ("rid", "kind", "dims", "prec", "arrival", "seed", "t_done", "result", "footprint")

    def __init__(self, rid, kind, dims, prec, arrival, seed):
        self.rid, self.kind, self.dims, self.prec = rid, kind, dims, prec
        self.arrival, self.seed = arrival, seed
        self.t_done = None
        self.result = None
        self.footprint = 0


def make_requests(count, rate, seed=8, frac_lu=0.1, precs=(128, 256, 512), gemm_range=(32, 1024),
                  lu_range=(64, 512)):
    """Seeded request mix; rate in requests per second (inf: all at time 0)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for rid in range(count):
        if math.isfinite(rate):
            t += rng.exponential(1.0 / rate)
        prec = int(rng.choice(precs))
        if rng.random() < frac_lu:
            n = int(round(math.exp(rng.uniform(math.log(lu_range[0]), math.log(lu_range[1])))))
            out.append(Request(rid, "lu", (n,), prec, t, int(rng.integers(1, 1 << 62))))
        else:
            d = [int(round(math.exp(rng.uniform(math.log(gemm_range[0]), math.log(gemm_range[1]))))) for _ in range(3)]
            out.append(Request(rid, "gemm", tuple(d), prec, t, int(rng.integers(1, 1 << 62))))
    return out


def words(rows, cols, prec):
    return (prec // 32 + 2) * rows * cols


def ws_words_estimate(m, l, n, prec, cutoff):
    """Workspace of a Winograd plan with peeling: at every level 4 + 4 operand
    sums and 7 products of the half sizes (the admission estimate)."""
    if min(m, l, n) <= cutoff:
        return 0
    h, g, w = m // 2, l // 2, n // 2
    return words(h, g, prec) * 4 + words(g, w, prec) * 4 + words(h, w, prec) * 7 + 7 * ws_words_estimate(h, g, w, prec, cutoff)


class Server:
    def __init__(self, slots=4, hbm_budget_gb=48.0, max_batch=32, algo=mp.WINOGRAD, cutoff=64, panel=64,
                 lu_cutoff=32, keep=None):
        import torch
        self.torch = torch
        self.slots = [torch.cuda.Stream() for _ in range(slots)]
        self.budget = hbm_budget_gb * 2 ** 30
        self.max_batch = max_batch
        self.algo, self.cutoff, self.panel, self.lu_cutoff = algo, cutoff, panel, lu_cutoff
        self.keep = keep or set()

    # footprint: operands + result + library workspace for that shape
    def footprint(self, r):
        if r.kind == "gemm":
            m, l, n = r.dims
            ws = ws_words_estimate(m, l, n, r.prec, self.cutoff)
            return 4 * (words(m, l, r.prec) + words(l, n, r.prec) + words(m, n, r.prec) + ws)
        n = r.dims[0]
        m2 = max(n - self.panel, 0)
        ws = ws_words_estimate(m2, self.panel, m2, r.prec, self.lu_cutoff) + words(m2, m2, r.prec)
        return 4 * (2 * words(n, n, r.prec) + 3 * words(n, 1, r.prec) + ws)

    def _launch(self, batch, stream):
        """Enqueue a batch on its stream; returns (tensors to keep alive, event)."""
        torch = self.torch
        keep = []
        with torch.cuda.stream(stream):
            if batch[0].kind == "gemm":
                prec = batch[0].prec
                As, Bs, Cs = [], [], []
                for r in batch:
                    m, l, n = r.dims
                    A, B, C = mp.empty(m, l, prec), mp.empty(l, n, prec), mp.empty(m, n, prec)
                    mp.mp_fill_uniform(m, l, prec, A, r.seed)
                    mp.mp_fill_uniform(l, n, prec, B, r.seed ^ 0x5555)
                    As.append(A), Bs.append(B), Cs.append(C)
                mp.mp_gemm_batched(prec, self.algo, self.cutoff, As, Bs, Cs)
                keep = list(zip(batch, Cs)) + [(None, t) for t in As + Bs]
            else:
                r = batch[0]
                n, prec = r.dims[0], r.prec
                A = mp.empty(n, n, prec)
                mp.mp_fill_uniform(n, n, prec, A, r.seed)
                ones = mp.empty(n, 1, prec)
                ones[prec // 32 - 1] = -2 ** 31                # mantissa 2^(p-1): top limb 0x80000000
                ones[prec // 32] = 1                            # exponent 1: the value 1
                x = mp.empty(n, 1, prec)
                mp.mp_gemm(n, n, 1, prec, mp.SIMPLE, 0, A, ones, x)   # b = A * ones
                piv = torch.zeros(n, dtype=torch.int32, device="cuda")
                info = torch.zeros(1, dtype=torch.int32, device="cuda")
                mp.mp_lu_async(n, prec, A, piv, info, self.panel, self.algo, self.lu_cutoff)
                mp.mp_lu_solve(n, prec, A, piv, x)
                keep = [(r, x), (None, A), (None, ones), (None, piv), (None, info)]
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
        return keep, ev

    def run(self, requests, poll_s=50e-6):
        torch = self.torch
        pending = sorted(requests, key=lambda r: r.arrival)
        for r in pending:
            r.footprint = self.footprint(r)
        waiting = []
        free = list(range(len(self.slots)))
        inflight = []                      # (slot, batch, keep, event, footprint)
        used = 0
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        nxt = 0
        done = 0
        peak = 0
        while done < len(pending):
            now = time.perf_counter() - t_start
            while nxt < len(pending) and pending[nxt].arrival <= now:
                waiting.append(pending[nxt])
                nxt += 1
            # retire finished batches
            still = []
            for slot, batch, keep, ev, fp in inflight:
                if ev.query():
                    t = ev0.elapsed_time(ev) * 1e-3
                    for r, tensor in keep:
                        if r is not None:
                            r.t_done = t
                            if r.rid in self.keep:
                                r.result = mp.to_host(tensor)
                    done += len(batch)
                    used -= fp
                    free.append(slot)
                else:
                    still.append((slot, batch, keep, ev, fp))
            inflight = still
            # admit
            while free and waiting:
                head = waiting[0]
                if head.kind == "lu":
                    batch = [head]
                else:
                    batch = [r for r in waiting if r.kind == "gemm" and r.prec == head.prec][: self.max_batch]
                fp = 0
                take = []
                for r in batch:
                    if used + fp + r.footprint <= self.budget or (not take and not inflight):
                        take.append(r)
                        fp += r.footprint
                if not take:
                    break
                for r in take:
                    waiting.remove(r)
                slot = free.pop()
                keep, ev = self._launch(take, self.slots[slot])
                inflight.append((slot, take, keep, ev, fp))
                used += fp
                peak = max(peak, used)
            if not (free and waiting):
                time.sleep(poll_s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        lat = np.array([r.t_done - r.arrival for r in pending]) * 1e3
        gemm_ops = sum(2.0 * r.dims[0] * r.dims[1] * r.dims[2] for r in pending if r.kind == "gemm")
        last = max(r.t_done for r in pending)
        return {
            "requests": len(pending), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "req_per_s": len(pending) / last,
            "gemm_2mln_per_s": gemm_ops / last, "wall_s": wall, "peak_admitted_gb": peak / 2 ** 30,
        }

    def alone(self, reqs):
        """Recompute the given requests one at a time; returns {rid: planes}."""
        out = {}
        for r in reqs:
            keep, ev = self._launch([r], self.slots[0])
            ev.synchronize()
            for rr, tensor in keep:
                if rr is not None:
                    out[rr.rid] = mp.to_host(tensor)
        return out


def saturated_rate(server, count=400, seed=9):
    reqs = make_requests(count, float("inf"), seed)
    st = server.run(reqs)
    return st["req_per_s"]


def main():
    ap = argparse.ArgumentParser(description="MP GEMM / LU request loop on one GPU")
    ap.add_argument("--requests", type=int, default=10000)
    ap.add_argument("--rate", type=float, default=0.0, help="arrivals per second (0: 0.8 x measured saturation)")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--check", type=int, default=32, help="requests recomputed alone and compared bit for bit")
    args = ap.parse_args()
    srv = Server(slots=args.slots)
    sat = saturated_rate(srv)
    rate = args.rate or 0.8 * sat
    reqs = make_requests(args.requests, rate, seed=8)
    rng = np.random.default_rng(3)
    chk = set(int(v) for v in rng.choice(len(reqs), size=min(args.check, len(reqs)), replace=False))
    srv.keep = chk
    st = srv.run(reqs)
    ref = srv.alone([r for r in reqs if r.rid in chk])
    same = sum(1 for r in reqs if r.rid in chk and np.array_equal(ref[r.rid], r.result))
    st.update({"saturated_req_per_s": sat, "rate": rate, "identical_alone_vs_mix": "%d/%d" % (same, len(chk))})
    print(json.dumps(st))


if __name__ == "__main__":
    main()
