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

Failure handling: a request whose footprint alone exceeds the budget is
refused at arrival (status "refused", it never reaches the device); a
request still waiting `queue_timeout_s` after its arrival is dropped
("timeout"); `cancel(rid)` drops a waiting request, or discards the result
of one already on the device ("cancelled"); a launch that raises marks the
requests of its batch "error" with the library's code and message, and the
loop goes on with the others.  Every request ends with one status.

The scheduler is independent of the device: it drives an executor (launch a
batch on a slot, poll its completion) and a clock, so it is tested on the CPU
with a fake executor and a fake clock; `GpuExecutor` is the real one.

`run()` returns p50 / p99 latency of the completed requests, throughput, the
classical-equivalent rate of the products and the count of every status.
The results of a sampled subset are kept so that `alone()` can recompute
them one at a time and compare them bit for bit.
"""

import argparse
import json
import math
import time

import numpy as np

OK, REFUSED, TIMEOUT, CANCELLED, ERROR = "ok", "refused", "timeout", "cancelled", "error"
E_NOMEM = -4                     # the library's MP_E_NOMEM: does not fit the memory budget


class Request:
    __slots__ = ("rid", "kind", "dims", "prec", "arrival", "seed", "t_done", "result", "footprint", "status",
                 "code", "error")

    def __init__(self, rid, kind, dims, prec, arrival, seed):
        self.rid, self.kind, self.dims, self.prec = rid, kind, dims, prec
        self.arrival, self.seed = arrival, seed
        self.t_done = None
        self.result = None
        self.footprint = 0
        self.status = None        # one of OK, REFUSED, TIMEOUT, CANCELLED, ERROR once finished
        self.code = 0             # library error code for ERROR / REFUSED
        self.error = ""


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


def footprint(r, cutoff=64, panel=64, lu_cutoff=32):
    """HBM bytes a request holds while it runs: operands, result and the
    library's workspace for its shape."""
    if r.kind == "gemm":
        m, l, n = r.dims
        ws = ws_words_estimate(m, l, n, r.prec, cutoff)
        return 4 * (words(m, l, r.prec) + words(l, n, r.prec) + words(m, n, r.prec) + ws)
    n = r.dims[0]
    m2 = max(n - panel, 0)
    ws = ws_words_estimate(m2, panel, m2, r.prec, lu_cutoff) + words(m2, m2, r.prec)
    return 4 * (2 * words(n, n, r.prec) + 3 * words(n, 1, r.prec) + ws)


class WallClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def sleep(self, dt):
        time.sleep(dt)


class GpuExecutor:
    """Launches batches through the library on `slots` HIP streams.  A launch
    returns a handle with done() (a GPU event query), t_done (seconds from the
    executor's start event to the batch's completion event, on the GPU clock)
    and results ({rid: planes} of the requests whose result was asked for)."""

    def __init__(self, slots=4, algo=None, cutoff=64, panel=64, lu_cutoff=32):
        import torch
        from . import mp
        self.torch, self.mp = torch, mp
        self.slots = [torch.cuda.Stream() for _ in range(slots)]
        self.algo = mp.WINOGRAD if algo is None else algo
        self.cutoff, self.panel, self.lu_cutoff = cutoff, panel, lu_cutoff
        self.ev0 = None

    def start(self):
        self.torch.cuda.synchronize()
        self.ev0 = self.torch.cuda.Event(enable_timing=True)
        self.ev0.record()

    def finish(self):
        self.torch.cuda.synchronize()

    def nslots(self):
        return len(self.slots)

    def launch(self, batch, slot, keep):
        torch, mp = self.torch, self.mp
        stream = self.slots[slot]
        held = []
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
                outs = list(zip(batch, Cs))
                held = As + Bs
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
                outs = [(r, x)]
                held = [A, ones, piv, info]
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
        return _GpuHandle(self, ev, outs, held, keep)


class _GpuHandle:
    def __init__(self, ex, ev, outs, held, keep):
        self.ex, self.ev, self.outs, self.held, self.keep = ex, ev, outs, held, keep
        self.t_done = None
        self.results = {}

    def done(self):
        if not self.ev.query():
            return False
        self.t_done = self.ex.ev0.elapsed_time(self.ev) * 1e-3
        for r, t in self.outs:
            if r.rid in self.keep:
                self.results[r.rid] = self.ex.mp.to_host(t)
        self.outs = self.held = None
        return True


class Server:
    def __init__(self, slots=4, hbm_budget_gb=48.0, max_batch=32, algo=None, cutoff=64, panel=64, lu_cutoff=32,
                 keep=None, queue_timeout_s=None, executor=None, clock=None):
        self.executor = executor if executor is not None else GpuExecutor(slots, algo, cutoff, panel, lu_cutoff)
        self.clock = clock
        self.budget = hbm_budget_gb * 2 ** 30
        self.max_batch = max_batch
        self.cutoff, self.panel, self.lu_cutoff = cutoff, panel, lu_cutoff
        self.keep = keep or set()
        self.queue_timeout_s = queue_timeout_s
        self._cancel = set()
        self.waited_for_memory = 0        # admissions that had to wait for memory to free up

    def footprint(self, r):
        return footprint(r, self.cutoff, self.panel, self.lu_cutoff)

    def cancel(self, rid):
        """Drop request rid if it is still waiting; discard its result if it
        is already on the device.  Takes effect at the loop's next pass."""
        self._cancel.add(rid)

    def run(self, requests, poll_s=50e-6, on_pass=None):
        """Serve every request; returns the statistics.  on_pass(server, now)
        is called once per loop pass (used by tests to cancel at a given time)."""
        ex = self.executor
        pending = sorted(requests, key=lambda r: r.arrival)
        for r in pending:
            r.footprint = self.footprint(r)
            r.status, r.t_done, r.result = None, None, None
        waiting = []
        free = list(range(ex.nslots()))
        inflight = []                      # (slot, batch, handle, footprint)
        used = 0
        peak = 0
        # the executor's start mark (a GPU event after a device synchronisation)
        # and the arrival clock's zero are taken together
        ex.start()
        clock = self.clock or WallClock()
        nxt = 0
        finished = 0

        def finish(r, status, t=None, code=0, msg=""):
            nonlocal finished
            r.status, r.code, r.error = status, code, msg
            if t is not None:
                r.t_done = t
            finished += 1

        while finished < len(pending):
            now = clock.now()
            if on_pass is not None:
                on_pass(self, now)
            while nxt < len(pending) and pending[nxt].arrival <= now:
                r = pending[nxt]
                nxt += 1
                if r.footprint > self.budget:
                    finish(r, REFUSED, now, E_NOMEM, "footprint %d bytes above the %d-byte budget"
                           % (r.footprint, self.budget))
                else:
                    waiting.append(r)
            # cancellations and queue timeouts of waiting requests
            if self._cancel or self.queue_timeout_s is not None:
                keep_w = []
                for r in waiting:
                    if r.rid in self._cancel:
                        finish(r, CANCELLED, now)
                    elif self.queue_timeout_s is not None and now - r.arrival > self.queue_timeout_s:
                        finish(r, TIMEOUT, now)
                    else:
                        keep_w.append(r)
                waiting = keep_w
            # retire finished batches
            still = []
            for slot, batch, h, fp in inflight:
                if h.done():
                    for r in batch:
                        if r.rid in self._cancel:
                            finish(r, CANCELLED, h.t_done)
                        else:
                            r.result = h.results.get(r.rid)
                            finish(r, OK, h.t_done)
                    used -= fp
                    free.append(slot)
                else:
                    still.append((slot, batch, h, fp))
            inflight = still
            # admit
            launched = False
            while free and waiting:
                head = waiting[0]
                if head.kind == "lu":
                    batch = [head]
                else:
                    batch = [r for r in waiting if r.kind == "gemm" and r.prec == head.prec][: self.max_batch]
                fp = 0
                take = []
                for r in batch:
                    if used + fp + r.footprint <= self.budget:
                        take.append(r)
                        fp += r.footprint
                if not take or take[0] is not head:
                    # the head does not fit now: wait for memory (arrival order is kept)
                    self.waited_for_memory += 1 if inflight else 0
                    if not inflight:          # nothing running can free memory: cannot happen (refused above)
                        finish(head, REFUSED, now, E_NOMEM, "does not fit the budget")
                        waiting.remove(head)
                        continue
                    break
                for r in take:
                    waiting.remove(r)
                slot = free.pop()
                try:
                    h = ex.launch(take, slot, self.keep)
                except Exception as e:            # a failed launch fails its own batch only
                    code = getattr(e, "code", -1)
                    for r in take:
                        finish(r, ERROR, clock.now(), code, str(e))
                    free.append(slot)
                    continue
                inflight.append((slot, take, h, fp))
                used += fp
                peak = max(peak, used)
                launched = True
            if finished < len(pending) and not launched:
                clock.sleep(poll_s)
        ex.finish()
        wall = clock.now()
        done = [r for r in pending if r.status == OK]
        lat = np.array([r.t_done - r.arrival for r in done]) * 1e3 if done else np.zeros(1)
        gemm_ops = sum(2.0 * r.dims[0] * r.dims[1] * r.dims[2] for r in done if r.kind == "gemm")
        last = max([r.t_done for r in done] + [1e-9])
        counts = {s: sum(1 for r in pending if r.status == s) for s in (OK, REFUSED, TIMEOUT, CANCELLED, ERROR)}
        return {
            "requests": len(pending), "completed": counts[OK], "refused": counts[REFUSED],
            "timed_out": counts[TIMEOUT], "cancelled": counts[CANCELLED], "failed": counts[ERROR],
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "req_per_s": counts[OK] / last,
            "gemm_2mln_per_s": gemm_ops / last, "wall_s": wall, "peak_admitted_gb": peak / 2 ** 30,
            "waited_for_memory": self.waited_for_memory,
        }

    def alone(self, reqs):
        """Recompute the given requests one at a time; returns {rid: planes}."""
        ex = self.executor
        ex.start()
        out = {}
        keep = set(r.rid for r in reqs)
        for r in reqs:
            h = ex.launch([r], 0, keep)
            while not h.done():
                time.sleep(50e-6)
            out.update(h.results)
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
    ap.add_argument("--budget-gb", type=float, default=48.0)
    ap.add_argument("--queue-timeout-s", type=float, default=None)
    ap.add_argument("--check", type=int, default=32, help="requests recomputed alone and compared bit for bit")
    args = ap.parse_args()
    srv = Server(slots=args.slots, hbm_budget_gb=args.budget_gb, queue_timeout_s=args.queue_timeout_s)
    sat = saturated_rate(srv)
    rate = args.rate or 0.8 * sat
    reqs = make_requests(args.requests, rate, seed=8)
    rng = np.random.default_rng(3)
    chk = set(int(v) for v in rng.choice(len(reqs), size=min(args.check, len(reqs)), replace=False))
    srv.keep = chk
    st = srv.run(reqs)
    ok = [r for r in reqs if r.rid in chk and r.status == OK]
    ref = srv.alone(ok)
    same = sum(1 for r in ok if np.array_equal(ref[r.rid], r.result))
    st.update({"saturated_req_per_s": sat, "rate": rate, "identical_alone_vs_mix": "%d/%d" % (same, len(ok))})
    print(json.dumps(st))


if __name__ == "__main__":
    main()
