"""The serving loop's scheduling and failure handling, on the CPU with a fake
engine (no GPU): admission by footprint, continuous batching, errors."""
import threading
import time

import numpy as np
import pytest

from paper_2412_11081_amd.serve import Engine, Request, Server, poisson_arrivals, replay


class FakeEngine(Engine):
    """payload = dict(bytes=..., secs=..., fail_admit=bool, fail_run=bool, value=x)."""

    def __init__(self):
        self.lock = threading.Lock()
        self.held = 0
        self.max_held = 0
        self.runs = []

    def estimate(self, p):
        if p.get("fail_estimate"):
            raise ValueError("bad request")
        return p["bytes"]

    def admit(self, p):
        if p.get("fail_admit"):
            raise RuntimeError("invalid tensors")
        with self.lock:
            self.held += p["bytes"]
            self.max_held = max(self.max_held, self.held)
        return p, p["bytes"]

    def run(self, handles):
        self.runs.append(len(handles))
        time.sleep(max(h["secs"] for h in handles))
        if any(h.get("fail_run") for h in handles):
            raise RuntimeError("device error")
        return [h["value"] * 2 for h in handles]

    def release(self, h):
        with self.lock:
            self.held -= h["bytes"]


def _server(eng, budget=100, max_batch=4, workers=2):
    return Server(eng, hbm_budget=budget, max_batch=max_batch, workers=workers)


def test_every_request_gets_its_own_result():
    eng = FakeEngine()
    srv = _server(eng)
    reqs = [srv.submit(Request(i, dict(bytes=10, secs=0.01, value=i))) for i in range(20)]
    assert srv.drain(timeout=30)
    srv.close()
    assert all(r.error is None and r.result == 2 * r.rid for r in reqs)
    assert eng.held == 0


def test_admission_never_exceeds_budget():
    eng = FakeEngine()
    srv = _server(eng, budget=50)
    for i in range(30):
        srv.submit(Request(i, dict(bytes=20, secs=0.005, value=i)))
    assert srv.drain(timeout=30)
    srv.close()
    assert eng.max_held <= 50 and srv.max_used <= 50
    assert srv.stats()["completed"] == 30


def test_request_over_budget_is_rejected_others_proceed():
    eng = FakeEngine()
    srv = _server(eng, budget=50)
    big = srv.submit(Request(0, dict(bytes=51, secs=0.0, value=0)))
    small = srv.submit(Request(1, dict(bytes=10, secs=0.0, value=1)))
    assert srv.drain(timeout=10)
    srv.close()
    assert big.error and "budget" in big.error
    assert small.error is None and small.result == 2


def test_failed_admission_and_failed_batch_are_reported():
    eng = FakeEngine()
    srv = _server(eng, max_batch=1, workers=1)
    a = srv.submit(Request(0, dict(bytes=10, secs=0.0, value=0, fail_admit=True)))
    b = srv.submit(Request(1, dict(bytes=10, secs=0.0, value=1, fail_run=True)))
    c = srv.submit(Request(2, dict(bytes=10, secs=0.0, value=2)))
    d = srv.submit(Request(3, dict(fail_estimate=True)))
    assert srv.drain(timeout=10)
    srv.close()
    assert a.error and "admission" in a.error
    assert b.error and "evaluation" in b.error
    assert c.error is None and c.result == 4
    assert d.error and "estimate" in d.error
    assert eng.held == 0 and srv.max_used <= 100


def test_continuous_batching_groups_requests_that_arrive_during_a_run():
    eng = FakeEngine()
    srv = _server(eng, budget=1000, max_batch=8, workers=1)
    first = srv.submit(Request(0, dict(bytes=1, secs=0.2, value=0)))
    time.sleep(0.05)                       # the first batch is running
    rest = [srv.submit(Request(i, dict(bytes=1, secs=0.01, value=i))) for i in range(1, 6)]
    assert srv.drain(timeout=10)
    srv.close()
    assert eng.runs[0] == 1 and max(eng.runs) >= 5       # the late arrivals share one batch
    assert all(r.error is None for r in [first] + rest)


def test_poisson_replay_and_latency_stats():
    eng = FakeEngine()
    srv = _server(eng, budget=200, max_batch=4, workers=2)
    arr = poisson_arrivals(40, rate=400.0, seed=3)
    assert np.all(np.diff(arr) > 0)
    reqs = replay(srv, [dict(bytes=5, secs=0.002, value=i) for i in range(40)], arr)
    assert srv.drain(timeout=30)
    srv.close()
    st = srv.stats()
    assert st["completed"] == 40 and st["failed"] == 0
    assert 0 < st["p50_s"] <= st["p99_s"]
    assert all(r.t_submit <= r.t_done for r in reqs)


def test_batching_window_gathers_requests_admitted_close_together():
    """With a window, a free worker waits for the requests being admitted
    (up to max_batch or the window) instead of taking the first one alone;
    without one it takes whatever is ready."""
    sizes = {}
    for window in (0.0, 0.05):
        eng = FakeEngine()
        srv = Server(eng, hbm_budget=1000, max_batch=6, workers=1, admitters=4, window=window)
        reqs = [srv.submit(Request(i, dict(bytes=10, secs=0.02, value=i))) for i in range(12)]
        assert srv.drain(timeout=30)
        srv.close()
        assert all(r.error is None for r in reqs)
        sizes[window] = list(srv.batches)
    assert sizes[0.05] == [6, 6], sizes
    assert len(sizes[0.0]) > 2, sizes
