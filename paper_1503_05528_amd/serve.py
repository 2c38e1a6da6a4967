"""Continuous-batching inpainting server over libvi's batches.

Requests (a video, its occlusion mask and method parameters) arrive at any
time.  A scheduler thread

  * admits queued requests, oldest first, while the batch has a free slot and
    the request's device footprint (vi_footprint_bytes) fits in the free part
    of the HBM budget;
  * keeps every admitted request's pyramid, shift maps and iterate resident
    in its libvi context;
  * advances all admitted requests together, one EM iteration each per
    vi_batch_step (one captured graph launch), so requests that arrive while
    others run join the running batch at the next step;
  * hands each finished result back through a Future, frees its context and
    its share of the budget, and records its latency (arrival to result).

Several lanes can run side by side: each lane is its own batch, on its own
stream, driven by its own thread, and requests are routed to a lane by a
size class, so the EM iterations of a few large clips and of many small
clips overlap on the device instead of small clips waiting for every
iteration of a large one.  All lanes share one HBM budget.

The scheduler is written against a small engine interface (make / step /
output / release / footprint) so that its admission, queueing, cancellation
and failure-isolation logic can be exercised without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from concurrent.futures import Future
from typing import Any, Callable


@dataclasses.dataclass
class Request:
    video: Any  # uint8 [T][H][W][3] (numpy or torch)
    mask: Any  # uint8 [T][H][W]
    params: dict
    arrival: float = 0.0
    rid: int = 0
    hole_fraction: float = 0.05


@dataclasses.dataclass
class Record:
    rid: int
    arrival: float
    admitted: float
    finished: float
    ok: bool

    @property
    def latency(self):
        return self.finished - self.arrival


class Engine:
    """What the scheduler needs from an execution backend."""

    def footprint(self, req: Request) -> int:
        raise NotImplementedError

    def make(self, req: Request):
        """Create the request's resident state and add it to the running
        batch; returns a handle."""
        raise NotImplementedError

    def step(self) -> None:
        """Advance every admitted request by one step."""
        raise NotImplementedError

    def done(self, h) -> bool:
        raise NotImplementedError

    def output(self, h):
        raise NotImplementedError

    def release(self, h) -> None:
        raise NotImplementedError


class GpuEngine(Engine):
    """libvi batches on one GPU."""

    def __init__(self, tune=None, device: str = "cuda:0"):
        import torch
        from . import vi
        self.torch = torch
        self.vi = vi
        self.device = torch.device(device)
        # a stream of its own so that lanes overlap on the device
        self.stream = torch.cuda.Stream(device=self.device)
        self.batch = vi.Batch(tune=tune, stream=self.stream)

    def footprint(self, req):
        T, H, W = req.mask.shape[:3]
        p = self.vi.default_params(**req.params)
        return self.vi.footprint_bytes(p, W, H, T, req.hole_fraction)

    def make(self, req):
        torch = self.torch
        v = req.video if isinstance(req.video, torch.Tensor) else torch.from_numpy(req.video)
        m = req.mask if isinstance(req.mask, torch.Tensor) else torch.from_numpy(req.mask)
        clip = self.vi.Clip(v.to(self.device), m.to(self.device), **req.params)
        self.batch.add(clip)
        return clip

    def step(self):
        self.batch.step()

    def done(self, h):
        return h.done()

    def output(self, h):
        return h.output().cpu().numpy()

    def release(self, h):
        try:
            self.batch.remove(h)
        finally:
            h.close()

    def close(self):
        self.batch.close()


class _Lane:
    def __init__(self, engine: Engine):
        self.engine = engine
        self.queue: collections.deque = collections.deque()
        self.running: dict = {}  # handle -> (req, future, bytes, admitted)
        self.thread: threading.Thread | None = None
        self.steps = 0


class Server:
    """engine: one Engine, or a list of engines (lanes); route(req) -> lane
    index picks the lane of a request (default: lane 0)."""

    def __init__(self, engine, hbm_budget: int, max_slots: int = 64,
                 route: Callable[[Request], int] | None = None,
                 clock: Callable[[], float] = time.perf_counter):
        engines = engine if isinstance(engine, (list, tuple)) else [engine]
        self.lanes = [_Lane(e) for e in engines]
        self.engine = engines[0]
        self.route = route or (lambda req: 0)
        self.budget = int(hbm_budget)
        self.max_slots = max_slots
        self.clock = clock
        self._lock = threading.Condition()
        self.used = 0
        self.records: list[Record] = []
        self._stop = False
        self._next_id = 0
        self.max_admitted_bytes = 0
        self.max_running = 0

    @property
    def steps(self):
        return sum(l.steps for l in self.lanes)

    # ---------------------------------------------------------------- API
    def submit(self, req: Request) -> Future:
        fut: Future = Future()
        with self._lock:
            req.rid = self._next_id
            self._next_id += 1
            if not req.arrival:
                req.arrival = self.clock()
            lane = self.lanes[min(len(self.lanes) - 1, max(0, int(self.route(req))))]
            lane.queue.append((req, fut))
            self._lock.notify_all()
        return fut

    def start(self):
        for i, lane in enumerate(self.lanes):
            lane.thread = threading.Thread(target=self._loop, args=(lane,),
                                           name=f"vi-server-{i}", daemon=True)
            lane.thread.start()

    def stop(self, drain: bool = True):
        with self._lock:
            if not drain:
                for lane in self.lanes:
                    for req, fut in lane.queue:
                        fut.cancel()
                    lane.queue.clear()
            self._stop = True
            self._lock.notify_all()
        for lane in self.lanes:
            if lane.thread:
                lane.thread.join()

    def queued(self) -> int:
        with self._lock:
            return sum(len(l.queue) for l in self.lanes)

    def running(self) -> int:
        return sum(len(l.running) for l in self.lanes)

    # ---------------------------------------------------------------- loop
    def _admit(self, lane: _Lane):
        while True:
            with self._lock:
                if not lane.queue or self.running() >= self.max_slots:
                    return
                req, fut = lane.queue[0]
                if fut.cancelled():
                    lane.queue.popleft()
                    continue
                try:
                    need = lane.engine.footprint(req)
                except Exception as e:  # invalid request: fail it alone
                    lane.queue.popleft()
                    fut.set_exception(e)
                    t = self.clock()
                    self.records.append(Record(req.rid, req.arrival, t, t, False))
                    continue
                if need <= 0 or need > self.budget:
                    lane.queue.popleft()
                    fut.set_exception(ValueError(
                        f"request {req.rid} needs {need} bytes; the budget is {self.budget}"))
                    continue
                if self.used + need > self.budget:
                    return  # oldest first: wait until memory frees up
                lane.queue.popleft()
                fut.set_running_or_notify_cancel()
                self.used += need  # reserved before the (slow) creation
            t = self.clock()
            try:
                h = lane.engine.make(req)
            except Exception as e:  # e.g. no hole-free patch: this request fails alone
                with self._lock:
                    self.used -= need
                fut.set_exception(e)
                self.records.append(Record(req.rid, req.arrival, t, self.clock(), False))
                continue
            with self._lock:
                lane.running[h] = (req, fut, need, t)
                self.max_admitted_bytes = max(self.max_admitted_bytes, self.used)
                self.max_running = max(self.max_running, self.running())

    def _retire(self, lane: _Lane):
        for h in list(lane.running):
            if not lane.engine.done(h):
                continue
            req, fut, need, t_adm = lane.running[h]
            try:
                out = lane.engine.output(h)
                ok = True
            except Exception as e:
                out, ok = e, False
            # the result is in host memory: it is handed over before the
            # release, which waits for the work the lane's other jobs queued
            t = self.clock()
            self.records.append(Record(req.rid, req.arrival, t_adm, t, ok))
            if ok:
                fut.set_result(out)
            else:
                fut.set_exception(out)
            try:
                lane.engine.release(h)
            finally:
                with self._lock:
                    del lane.running[h]
                    self.used -= need
                    self._lock.notify_all()

    def _loop(self, lane: _Lane):
        while True:
            self._admit(lane)
            if lane.running:
                try:
                    lane.engine.step()
                    lane.steps += 1
                except Exception as e:
                    # a failing step fails the requests that were in it
                    for h, (req, fut, need, t_adm) in list(lane.running.items()):
                        lane.engine.release(h)
                        with self._lock:
                            self.used -= need
                        fut.set_exception(e)
                        self.records.append(Record(req.rid, req.arrival, t_adm, self.clock(),
                                                   False))
                    with self._lock:
                        lane.running.clear()
                self._retire(lane)
                continue
            with self._lock:
                if self._stop and not lane.queue:
                    return
                if not lane.queue or self.used > 0:
                    self._lock.wait(timeout=0.02)

    # ---------------------------------------------------------------- stats
    def latency_stats(self):
        lat = sorted(r.latency for r in self.records if r.ok)
        if not lat:
            return {}

        def pct(q):
            return lat[min(len(lat) - 1, max(0, int(round(q * (len(lat) - 1)))))]
        return {"n": len(lat), "p50_s": pct(0.50), "p99_s": pct(0.99), "max_s": lat[-1],
                "mean_s": sum(lat) / len(lat)}


def fifo_latencies(arrivals, service):
    """Latencies of serial first-in-first-out execution: each request starts
    when it has arrived and the previous one has finished."""
    t = 0.0
    out = []
    for a, s in zip(arrivals, service):
        start = max(t, a)
        t = start + s
        out.append(t - a)
    return out


def percentile(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, max(0, int(round(q * (len(xs) - 1)))))]
