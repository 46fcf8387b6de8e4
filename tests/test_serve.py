"""CPU tests of the serving scheduler (admission by HBM footprint, continuous
batching, failure isolation), driven by a fake backend with a simulated
clock.  The GPU path of the same scheduler is tested in test_gpu_serve.py."""
import numpy as np
import pytest

from paper_2109_14704_amd import serve


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeBackend:
    """Steps complete `delay` simulated seconds after launch; the 'result' of a
    request is a function of its own operands only, so mixing requests up is
    visible.  fail_on: launch indices that raise."""

    def __init__(self, clock, delay=1.0, fail_on=()):
        self.clock, self.delay, self.fail_on = clock, delay, set(fail_on)
        self.launches = 0
        self.groups = []
        self.inflight = 0          # steps launched and not yet released
        self.max_inflight = 0

    def launch(self, batch, slot=0):
        k = self.launches
        self.launches += 1
        if k in self.fail_on:
            raise RuntimeError("injected failure on launch %d" % k)
        self.groups.append([(key, [r.rid for r in rs]) for key, rs in batch])
        self.inflight += 1
        self.max_inflight = max(self.max_inflight, self.inflight)
        return {"t": self.clock() + self.delay, "batch": batch}

    def poll(self, h):
        return True if self.clock() >= h["t"] else None

    def collect(self, h, reqs):
        for r in reqs:
            r.result = int(np.sum(r.c)) * 31 + int(np.sum(r.d))

    def release(self, h):
        self.inflight -= 1


def make_req(i, arrival, log_n=14, level=4):
    rng = np.random.default_rng(i)
    return serve.Request(i, arrival, log_n, level, rng.integers(0, 1000, 8), rng.integers(0, 1000, 8))


def drive(s, clock, reqs, dt=0.25, limit=1000):
    pending = sorted(reqs, key=lambda r: r.arrival)
    steps = 0
    while (pending or not s.idle()) and steps < limit:
        while pending and pending[0].arrival <= clock.t:
            s.submit(pending.pop(0))
        s.tick()
        clock.t += dt
        steps += 1
    return steps


def test_budget_is_never_exceeded_and_everything_completes():
    clock = Clock()
    be = FakeBackend(clock)
    fp = serve.footprint(14, 4)
    s = serve.Scheduler(be, budget_bytes=3 * fp, streams=2, clock=clock)
    reqs = [make_req(i, 0.0) for i in range(10)]
    drive(s, clock, reqs)
    assert all(r.state == "done" for r in reqs)
    assert s.max_reserved <= 3 * fp and s.reserved == 0
    for r in reqs:
        assert r.result == int(np.sum(r.c)) * 31 + int(np.sum(r.d))


def test_continuous_batching_admits_arrivals_between_steps():
    clock = Clock()
    be = FakeBackend(clock, delay=2.0)
    s = serve.Scheduler(be, budget_bytes=10 ** 12, streams=2, clock=clock)
    reqs = [make_req(i, 0.5 * i, log_n=14 + i % 2, level=4 + i % 3) for i in range(12)]
    drive(s, clock, reqs)
    assert all(r.state == "done" for r in reqs)
    # late arrivals were launched in later steps while earlier steps were in flight
    assert be.launches >= 3
    # each launched group holds one (N, level)
    for step in be.groups:
        for (ln, lvl), rids in step:
            assert all((reqs[i].log_n, reqs[i].level) == (ln, lvl) for i in rids)
    # at most `streams` steps in flight at once, and the limit was reached:
    # arrivals every 0.5 s against 2 s steps keep two steps in flight
    assert be.max_inflight == 2 and be.inflight == 0


def test_full_queue_keeps_two_steps_in_flight():
    """All requests at t = 0 with the budget full: each step takes at most half
    the budget, so the second step is launched while the first runs."""
    clock = Clock()
    be = FakeBackend(clock, delay=2.0)
    fp = serve.footprint(14, 4)
    s = serve.Scheduler(be, budget_bytes=4 * fp, streams=2, clock=clock)
    reqs = [make_req(i, 0.0) for i in range(8)]
    for r in reqs:
        s.submit(r)
    s.tick()                              # admits 4, launches 2 + 2
    assert be.launches == 2 and be.inflight == 2
    assert [sum(len(rids) for _, rids in step) for step in be.groups] == [2, 2]
    drive(s, clock, [])
    assert all(r.state == "done" for r in reqs) and s.reserved == 0
    assert be.launches == 4 and be.max_inflight == 2


def test_oversized_request_is_rejected_not_blocking():
    clock = Clock()
    be = FakeBackend(clock)
    s = serve.Scheduler(be, budget_bytes=serve.footprint(14, 4), clock=clock)
    big = make_req(0, 0.0, log_n=16, level=24)
    small = make_req(1, 0.0)
    drive(s, clock, [big, small])
    assert big.state == "rejected" and "exceeds" in big.error
    assert small.state == "done"


def test_failed_launch_fails_only_its_requests_and_frees_memory():
    clock = Clock()
    be = FakeBackend(clock, delay=1.0, fail_on={1})
    s = serve.Scheduler(be, budget_bytes=10 ** 12, streams=1, clock=clock)
    reqs = [make_req(i, 1.1 * i) for i in range(6)]
    drive(s, clock, reqs)
    failed = [r for r in reqs if r.state == "failed"]
    assert failed and all("injected" in r.error for r in failed)
    assert all(r.state in ("done", "failed") for r in reqs)
    assert any(r.state == "done" for r in reqs)
    assert s.reserved == 0


def test_cancel_before_launch():
    clock = Clock()
    be = FakeBackend(clock, delay=5.0)
    s = serve.Scheduler(be, budget_bytes=10 ** 12, streams=1, clock=clock)
    a, b = make_req(0, 0.0), make_req(1, 0.0)
    s.submit(a)
    s.tick()                      # a launched
    s.submit(b)
    assert s.cancel(b)
    assert not s.cancel(a)        # already launched
    drive(s, clock, [])
    assert a.state == "done" and b.state == "cancelled" and s.reserved == 0


def test_results_identical_alone_and_in_the_mix():
    def run(reqs):
        clock = Clock()
        s = serve.Scheduler(FakeBackend(clock), budget_bytes=10 ** 12, clock=clock)
        drive(s, clock, reqs)
        return {r.rid: r.result for r in reqs}
    mix = run([make_req(i, 0.1 * i, 14 + i % 3, 4 + i % 5) for i in range(15)])
    for i in range(15):
        alone = run([make_req(i, 0.0, 14 + i % 3, 4 + i % 5)])
        assert alone[i] == mix[i]


def test_latency_stats():
    reqs = [make_req(i, 0.0) for i in range(100)]
    for i, r in enumerate(reqs):
        r.state, r.t_done = "done", (i + 1) * 1e-3
    st = serve.latency_stats(reqs)
    assert st["completed"] == 100 and st["p50_ms"] == pytest.approx(50.5) and st["p99_ms"] == pytest.approx(99.01)
