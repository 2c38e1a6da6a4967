"""Scheduler logic of the continuous-batching server on a fake CPU engine:
admission by footprint within the budget, oldest-first queueing, requests
joining a running batch, failure isolation, cancellation, latency records,
and the serial first-in-first-out reference."""
import threading
import time

import numpy as np
import pytest

from paper_1503_05528_amd.serve import Engine, Request, Server, fifo_latencies, percentile


class FakeEngine(Engine):
    """Each request takes params['iters'] steps; params['bytes'] of memory;
    params['fail'] makes creation fail."""

    def __init__(self):
        self.live = {}
        self.step_sizes = []
        self.created = []

    def footprint(self, req):
        if req.params.get("bad_footprint"):
            raise ValueError("bad request")
        return req.params["bytes"]

    def make(self, req):
        if req.params.get("fail"):
            raise RuntimeError("creation failed")
        h = object()
        self.live[h] = [req.params["iters"], req.rid]
        self.created.append(req.rid)
        return h

    def step(self):
        self.step_sizes.append(len(self.live))
        for v in self.live.values():
            v[0] -= 1
        time.sleep(0.001)

    def done(self, h):
        return self.live[h][0] <= 0

    def output(self, h):
        return ("result", self.live[h][1])

    def release(self, h):
        del self.live[h]


def req(iters=3, nbytes=10, **kw):
    p = dict(iters=iters, bytes=nbytes)
    p.update(kw)
    return Request(video=None, mask=np.zeros((1, 1, 1), np.uint8), params=p)


def test_results_and_budget():
    eng = FakeEngine()
    srv = Server(eng, hbm_budget=25, max_slots=8)
    futs = [srv.submit(req(iters=2 + i % 3)) for i in range(10)]
    srv.start()
    outs = [f.result(timeout=10) for f in futs]
    srv.stop()
    assert outs == [("result", i) for i in range(10)]
    assert srv.max_admitted_bytes <= 25
    assert srv.max_running == 2  # 2 x 10 bytes fit in 25
    assert eng.created == list(range(10))  # oldest first
    st = srv.latency_stats()
    assert st["n"] == 10 and st["p99_s"] >= st["p50_s"] > 0


def test_slots_limit_and_joining_running_batch():
    eng = FakeEngine()
    srv = Server(eng, hbm_budget=10 ** 9, max_slots=3)
    srv.start()
    first = [srv.submit(req(iters=40)) for _ in range(2)]
    time.sleep(0.02)
    late = [srv.submit(req(iters=5)) for _ in range(3)]
    for f in first + late:
        f.result(timeout=10)
    srv.stop()
    assert srv.max_running == 3
    # the late requests ran in the same steps as the long ones
    assert max(eng.step_sizes) == 3
    rec = {r.rid: r for r in srv.records}
    assert all(rec[i].finished < rec[0].finished for i in (2, 3))


def test_failure_isolation_and_oversized():
    eng = FakeEngine()
    srv = Server(eng, hbm_budget=100, max_slots=4)
    good1 = srv.submit(req())
    bad = srv.submit(req(fail=True))
    huge = srv.submit(req(nbytes=1000))
    invalid = srv.submit(req(bad_footprint=True))
    good2 = srv.submit(req())
    srv.start()
    assert good1.result(timeout=10)[0] == "result"
    assert good2.result(timeout=10)[0] == "result"
    with pytest.raises(RuntimeError):
        bad.result(timeout=10)
    with pytest.raises(ValueError):
        huge.result(timeout=10)
    with pytest.raises(ValueError):
        invalid.result(timeout=10)
    srv.stop()
    assert eng.live == {}
    assert srv.used == 0


def test_cancel_before_admission():
    eng = FakeEngine()
    srv = Server(eng, hbm_budget=10, max_slots=1)
    a = srv.submit(req(iters=20))
    b = srv.submit(req(iters=2))
    assert b.cancel()
    srv.start()
    a.result(timeout=10)
    srv.stop()
    assert b.cancelled()
    assert eng.created == [0]


def test_stop_without_drain_cancels_queue():
    eng = FakeEngine()
    srv = Server(eng, hbm_budget=10, max_slots=1)
    srv.start()
    a = srv.submit(req(iters=30))
    rest = [srv.submit(req()) for _ in range(3)]
    time.sleep(0.01)
    srv.stop(drain=False)
    assert a.done()
    assert all(f.cancelled() or f.done() for f in rest)


def test_fifo_reference():
    # arrivals 0, 1, 1.5; services 2, 1, 1 -> finish 2, 3, 4
    lat = fifo_latencies([0.0, 1.0, 1.5], [2.0, 1.0, 1.0])
    assert lat == [2.0, 2.0, 2.5]
    assert percentile([3, 1, 2], 0.5) == 2


def test_two_lanes_overlap_and_share_budget():
    small, large = FakeEngine(), FakeEngine()
    srv = Server([small, large], hbm_budget=100, max_slots=16,
                 route=lambda r: 1 if r.params["bytes"] >= 50 else 0)
    srv.start()
    big = srv.submit(req(iters=200, nbytes=60))
    time.sleep(0.01)
    smalls = [srv.submit(req(iters=3, nbytes=10)) for _ in range(6)]
    for f in smalls:
        f.result(timeout=10)
    # the small requests finished while the large one was still running
    assert not big.done()
    big.result(timeout=20)
    srv.stop()
    assert srv.max_admitted_bytes <= 100
    assert large.created == [0] and small.created == [1, 2, 3, 4, 5, 6]
