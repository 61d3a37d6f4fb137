"""The serving loop's scheduler on the CPU: a fake executor (batches take a
time proportional to their work on a fake clock) and tiny memory budgets.
Checks admission by footprint (never above the budget, waiting for memory
when the head request does not fit, arrival order kept), refusal of a request
that can never fit, queue timeouts, cancellation of waiting and running
requests, and that a failing launch fails only its own batch."""

import pytest

from paper_1410_1599_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-4)


class FakeHandle:
    def __init__(self, ex, batch, t_end, keep):
        self.ex, self.batch, self.t_end, self.keep = ex, batch, t_end, keep
        self.t_done = None
        self.results = {}

    def done(self):
        if self.ex.clock.now() < self.t_end:
            return False
        if self.t_done is None:
            self.t_done = self.t_end
            self.results = {r.rid: ("result", r.rid) for r in self.batch if r.rid in self.keep}
            self.ex.running.remove(self)
        return True


class FakeExecutor:
    """A batch takes 1 ms per 10^6 classical multiply-adds (a solve: n^3)."""

    def __init__(self, clock, slots=2, fail_rids=()):
        self.clock, self.slots, self.fail_rids = clock, slots, set(fail_rids)
        self.running = []
        self.launched = []          # (time, [rids], footprint)
        self.max_concurrent_bytes = 0
        self.slot_busy = set()

    def start(self):
        pass

    def finish(self):
        pass

    def nslots(self):
        return self.slots

    def launch(self, batch, slot, keep):
        if any(r.rid in self.fail_rids for r in batch):
            raise RuntimeError("injected launch failure")
        work = sum(r.dims[0] * r.dims[1] * r.dims[2] if r.kind == "gemm" else r.dims[0] ** 3 for r in batch)
        h = FakeHandle(self, batch, self.clock.now() + 1e-3 * work / 1e6, keep)
        self.running.append(h)
        self.launched.append((self.clock.now(), [r.rid for r in batch], sum(r.footprint for r in batch)))
        self.max_concurrent_bytes = max(self.max_concurrent_bytes,
                                        sum(r.footprint for hh in self.running for r in hh.batch))
        return h


def gemm(rid, m, l, n, prec=256, t=0.0):
    return serve.Request(rid, "gemm", (m, l, n), prec, t, rid + 1)


def server(clock, ex, budget_bytes, **kw):
    return serve.Server(hbm_budget_gb=budget_bytes / 2 ** 30, executor=ex, clock=clock, **kw)


def test_request_above_budget_is_refused_and_never_launched():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    big, small = gemm(0, 400, 400, 400), gemm(1, 40, 40, 40)
    budget = (serve.footprint(small) + serve.footprint(big)) // 2
    assert serve.footprint(big) > budget >= serve.footprint(small)
    srv = server(clock, ex, budget)
    st = srv.run([big, small])
    assert big.status == serve.REFUSED and big.code == serve.E_NOMEM and "budget" in big.error
    assert small.status == serve.OK
    assert st["refused"] == 1 and st["completed"] == 1
    assert all(0 not in rids for _, rids, _ in ex.launched)


def test_admission_never_exceeds_budget_and_waits_for_memory():
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=4)
    reqs = [gemm(i, 200, 200, 200, prec=512) for i in range(12)]
    one = serve.footprint(reqs[0])
    srv = server(clock, ex, int(2.5 * one), max_batch=1)
    st = srv.run(reqs)
    assert st["completed"] == 12
    assert ex.max_concurrent_bytes <= int(2.5 * one)
    assert max(len(rids) for _, rids, _ in ex.launched) == 1
    assert st["waited_for_memory"] > 0 and st["peak_admitted_gb"] * 2 ** 30 <= 2.5 * one
    # arrival order: launches in rid order
    order = [rids[0] for _, rids, _ in ex.launched]
    assert order == sorted(order)


def test_batches_group_same_precision_products():
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=1)
    reqs = [gemm(i, 50, 50, 50, prec=(128 if i % 2 else 256), t=0.0) for i in range(8)]
    st = server(clock, ex, 1 << 40).run(reqs)
    assert st["completed"] == 8
    for _, rids, _ in ex.launched:
        assert len({reqs[r].prec for r in rids}) == 1
    assert max(len(rids) for _, rids, _ in ex.launched) > 1


def test_requests_arriving_meanwhile_join_later_batches():
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=2)
    reqs = [gemm(i, 300, 300, 300, t=0.005 * i) for i in range(10)]
    st = server(clock, ex, 1 << 40).run(reqs)
    assert st["completed"] == 10
    assert all(r.t_done >= r.arrival for r in reqs)
    # work was running while later requests arrived and were admitted
    assert any(t > 0 for t, _, _ in ex.launched[1:])


def test_queue_timeout_drops_waiting_requests():
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=1)
    reqs = [gemm(i, 500, 500, 500) for i in range(5)]      # 125 ms each
    srv = server(clock, ex, 1 << 40, max_batch=1, queue_timeout_s=0.2)
    st = srv.run(reqs)
    launched = {r for _, rids, _ in ex.launched for r in rids}
    for r in reqs:
        assert r.status in (serve.OK, serve.TIMEOUT)
        assert (r.status == serve.OK) == (r.rid in launched)
    assert st["timed_out"] >= 2 and st["completed"] >= 1
    assert st["completed"] + st["timed_out"] == 5


def test_cancel_waiting_and_running_requests():
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=1)
    reqs = [gemm(i, 400, 400, 400) for i in range(4)]
    srv = server(clock, ex, 1 << 40, max_batch=1, keep={0, 1, 2, 3})

    def on_pass(s, now):
        if now > 0.01:
            s.cancel(0)       # running by then
            s.cancel(3)       # still waiting

    st = srv.run(reqs, on_pass=on_pass)
    assert reqs[0].status == serve.CANCELLED and reqs[0].result is None
    assert reqs[3].status == serve.CANCELLED
    assert 3 not in {r for _, rids, _ in ex.launched for r in rids}
    assert reqs[1].status == reqs[2].status == serve.OK and reqs[1].result == ("result", 1)
    assert st["cancelled"] == 2 and st["completed"] == 2


def test_failing_launch_fails_only_its_batch():
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=2, fail_rids={2})
    reqs = [gemm(i, 60, 60, 60) for i in range(6)]
    srv = server(clock, ex, 1 << 40, max_batch=1)
    st = srv.run(reqs)
    assert reqs[2].status == serve.ERROR and "injected" in reqs[2].error and reqs[2].code == -1
    assert all(r.status == serve.OK for r in reqs if r.rid != 2)
    assert st["failed"] == 1 and st["completed"] == 5


def test_every_request_ends_with_one_status():
    clock = FakeClock()
    ex = FakeExecutor(clock, slots=3, fail_rids={7})
    reqs = serve.make_requests(60, 300.0, seed=4, gemm_range=(32, 400), lu_range=(64, 200))
    budget = sorted(serve.footprint(r) for r in reqs)[-3]     # the two largest can never fit
    srv = server(clock, ex, budget, queue_timeout_s=0.3)
    st = srv.run(reqs)
    assert all(r.status in (serve.OK, serve.REFUSED, serve.TIMEOUT, serve.CANCELLED, serve.ERROR) for r in reqs)
    assert sum(st[k] for k in ("completed", "refused", "timed_out", "cancelled", "failed")) == 60
    assert st["refused"] >= 1
    assert ex.max_concurrent_bytes <= budget


@pytest.mark.parametrize("kind", ["gemm", "lu"])
def test_footprint_counts_operands_result_and_workspace(kind):
    r = gemm(0, 256, 256, 256) if kind == "gemm" else serve.Request(0, "lu", (256,), 256, 0.0, 1)
    fp = serve.footprint(r)
    W = (256 // 32 + 2) * 4
    assert fp >= 3 * 256 * 256 * W if kind == "gemm" else fp >= 2 * 256 * 256 * W
