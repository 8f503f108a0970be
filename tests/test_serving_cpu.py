"""Scheduling logic of the continuous-batching loop, driven by a simulated
executor on a virtual clock (no GPU)."""

import numpy as np

from paper_2506_23775_amd.serving import ContinuousBatcher, Request, latency_stats


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, d):
        self.t += d


class FakeExec:
    """Each chunk occupies the request's stream for `chunk_time` seconds."""

    def __init__(self, clock, chunk_time=1.0):
        self.clock = clock
        self.chunk_time = chunk_time
        self.busy = {}
        self.max_concurrent = 0
        self.issue_log = []

    def footprint(self, req):
        return req.payload["bytes"]

    def admit(self, req):
        req.state["acc"] = 0.0
        return [(-1, i, 1) for i in range(req.payload["chunks"])]

    def idle(self, req):
        return self.clock.t >= self.busy.get(req.rid, -1.0)

    def issue(self, req, chunk, first=False):
        self.busy[req.rid] = self.clock.t + self.chunk_time
        req.state["acc"] += chunk[1] + 1
        running = sum(1 for v in self.busy.values() if v > self.clock.t)
        self.max_concurrent = max(self.max_concurrent, running)
        self.issue_log.append((self.clock.t, req.rid, chunk[1]))

    def wait_any(self, active):
        ts = [self.busy[r.rid] for r in active if self.busy.get(r.rid, -1) > self.clock.t]
        if ts:
            self.clock.t = min(ts)

    def finish(self, req):
        return {"f": req.state["acc"]}


def _reqs(spec):
    return [Request(rid=i, arrival=a, op=op, k=8, payload=dict(bytes=b, chunks=n))
            for i, (a, op, b, n) in enumerate(spec)]


def test_all_complete_and_budget_respected():
    clk = Clock()
    ex = FakeExec(clk)
    b = ContinuousBatcher(ex, hbm_budget=100, max_active=4, clock=clk, sleep=clk.sleep)
    rng = np.random.default_rng(0)
    spec = [(float(a), "hvp", int(rng.integers(10, 60)), int(rng.integers(1, 5)))
            for a in np.cumsum(rng.exponential(0.7, 25))]
    done = b.run(_reqs(spec))
    assert len(done) == 25
    assert b.peak_used <= 100
    for r in done:
        n = r.payload["chunks"]
        assert r.result["f"] == n * (n + 1) / 2          # every chunk exactly once
        assert r.t_done >= r.t_admit >= r.arrival
    assert ex.max_concurrent >= 2                          # work of several requests overlaps


def test_late_arrival_joins_running_batch():
    clk = Clock()
    ex = FakeExec(clk)
    b = ContinuousBatcher(ex, hbm_budget=100, max_active=4, clock=clk, sleep=clk.sleep)
    done = b.run(_reqs([(0.0, "f", 10, 6), (2.5, "grad", 10, 2)]))
    by = {r.rid: r for r in done}
    # the second request is admitted while the first still has chunks in flight
    assert by[1].t_admit < by[0].t_done
    assert by[1].t_done < by[0].t_done


def test_admission_waits_for_memory():
    clk = Clock()
    ex = FakeExec(clk)
    b = ContinuousBatcher(ex, hbm_budget=100, max_active=8, clock=clk, sleep=clk.sleep)
    done = b.run(_reqs([(0.0, "f", 70, 3), (0.1, "f", 50, 1), (0.2, "f", 20, 1)]))
    by = {r.rid: r for r in done}
    # request 1 (50 bytes) cannot start before request 0 (70 bytes) finishes,
    # and FIFO order keeps request 2 behind it
    assert by[1].t_admit >= by[0].t_done
    assert by[2].t_admit >= by[1].t_admit
    assert b.peak_used <= 100
    st = latency_stats(done)
    assert st["all"]["n"] == 3 and st["all"]["p99_ms"] >= st["all"]["p50_ms"]


def test_oversized_request_rejected():
    clk = Clock()
    b = ContinuousBatcher(FakeExec(clk), hbm_budget=10, clock=clk, sleep=clk.sleep)
    try:
        b.run(_reqs([(0.0, "f", 11, 1)]))
    except ValueError as e:
        assert "budget" in str(e)
    else:
        raise AssertionError("expected rejection")
