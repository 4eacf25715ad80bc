"""Continuous-batching server for landscape analyses.

Requests (a search space, its fitness on the GPU, a neighbourhood, d and p)
arrive over time.  The server

* admits a request once its estimated device footprint fits under an HBM
  budget (default: the device's free memory at start-up minus a reserve),
  queueing it otherwise;
* keeps built fitness flow graphs in a device-resident LRU cache keyed by the
  request's content key, so a repeated space with another d or p only reruns
  PageRank;
* adds admitted requests to one running batch (fl_batch_*): members join and
  leave between steps of a few sweeps, so short analyses are not held behind
  long ones;
* records, per request, the latency from arrival to a host-visible result;
* keeps Python's cyclic garbage collector from running inside the loop (a
  full collection over the live request and tensor objects stalls the loop
  for tens of milliseconds): automatic collection is paused while ``run``
  serves and the young generations are collected when the loop idles.

The GPU work goes through a backend object (``build``, ``plan_bytes``,
``member_bytes``, ``add``, ``step``, ``collect``, ``release``, plus ``plain``
for the one-at-a-time reference path), so the scheduling logic can be
exercised with any backend.
"""
from __future__ import annotations

import collections
import gc
import heapq
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Hashable


@dataclass(order=True)
class Request:
    arrival: float                        # seconds on the server clock
    rid: int
    key: Hashable = field(compare=False)  # content key of (space, fitness, neighbourhood)
    radix: tuple = field(compare=False, default=())
    fitness: Any = field(compare=False, default=None)   # device float32 tensor
    neighbourhood: str = field(compare=False, default="hamming")
    damping: float = field(compare=False, default=0.85)
    p: float = field(compare=False, default=0.05)


@dataclass
class Done:
    rid: int
    arrival: float
    finish: float
    score: float
    pagerank: Any
    minima: Any
    info: dict

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


def footprint_estimate(radix, words: int = 2) -> int:
    """Upper bound (bytes) of the device memory an analysis of a space with
    these radices holds: node map, fitness copy and raw-space x vectors
    (4 n_raw each, two x buffers), records, degrees, CSR, iterates."""
    n_raw = 1
    for r in radix:
        n_raw *= int(r)
    k = sum(int(r) - 1 for r in radix)           # Hamming neighbours per node
    per_node = 8 * words + 4 * 4 + 2 * 4 + 4 * max(k // 2, 1)
    return n_raw * (4 * 4) + n_raw * per_node // 2 + (1 << 20)


class GpuBackend:
    """The engine through the Python binding (one context, one batch)."""

    def __init__(self, ctx=None, sweeps_per_step: int = 16):
        from . import api
        self.api = api
        self.ctx = ctx or api.Context(0)
        self.batch = api.Batch(self.ctx)
        self.sweeps = sweeps_per_step

    def build(self, req: Request):
        plan = self.api.plan_create(self.ctx, req.radix, req.fitness, req.neighbourhood)
        words = int(plan.sizes.get("mask_words", 0))
        batchable = words > 0 and 4 * plan.sizes["n_raw"] < 2 ** 31
        return plan, batchable

    def plan_bytes(self, plan) -> int:
        s = plan.sizes
        n, n_raw, e = int(s["n_valid"]), int(s["n_raw"]), int(s["n_edges"])
        return n_raw * 16 + n * (8 * max(int(s["mask_words"]), 1) + 28) + 4 * e

    def member_bytes(self, plan) -> int:
        s = plan.sizes
        n, n_raw = int(s["n_valid"]), int(s["n_raw"])
        return 8 * n_raw + 8 * n + 24 * ((n + 255) // 256) + 80

    def add(self, plan, req: Request) -> None:
        self.batch.add(plan, req.damping, req.p, tag=req.rid)

    def step(self) -> int:
        return self.batch.step(self.sweeps)

    def collect(self):
        return [(tag, pr, mins, info) for tag, pr, mins, info in self.batch.collect()]

    def plain(self, plan, req: Request):
        pr, mins, info = self.api.execute(plan, req.damping, req.p)
        return pr, mins, info

    def release(self, plan) -> None:
        plan.close()

    def sync(self) -> None:
        import torch
        torch.cuda.synchronize()

    def close(self) -> None:
        self.batch.close()


class Server:
    """Continuous-batching scheduler (see the module docstring)."""

    def __init__(self, backend, hbm_budget: int, cache_budget: int | None = None,
                 clock: Callable[[], float] | None = None,
                 sleep: Callable[[float], None] | None = None, pause_gc: bool = True):
        self.backend = backend
        self.pause_gc = pause_gc
        self.hbm_budget = int(hbm_budget)
        self.cache_budget = int(cache_budget if cache_budget is not None else hbm_budget // 2)
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.cache: "collections.OrderedDict[Hashable, tuple]" = collections.OrderedDict()
        self.cache_bytes = 0
        self.in_use: dict = {}            # key -> running members using the cached plan
        self.reserved = 0                 # bytes of running members' plans not in the cache
        self.peak_bytes = 0
        self.queue: list = []             # admitted order: waiting requests
        self.running: dict = {}           # rid -> (req, key, plan, bytes, shared)
        self.done: list = []
        self.stats = collections.Counter()

    # -- memory accounting -------------------------------------------------
    def _held(self) -> int:
        return self.cache_bytes + self.reserved

    def _evict(self, need: int, keep=None) -> None:
        for key in list(self.cache):
            if self._held() + need <= self.hbm_budget:
                return
            if key == keep or self.in_use.get(key, 0) > 0:
                continue
            plan, nbytes, _ = self.cache.pop(key)
            self.cache_bytes -= nbytes
            self.backend.release(plan)
            self.stats["evicted"] += 1

    def _admit(self, req: Request) -> bool:
        """Build or reuse the request's plan and add it to the batch, if the
        budget allows; False leaves the request queued.  A plan that fits the
        cache budget is cached and shared (members running on one FFG keep
        their own iterate vectors); any other is owned by its request and
        released when the request finishes."""
        hit = self.cache.get(req.key)
        n_raw = 1
        for r in req.radix:
            n_raw *= int(r)
        need = 16 * n_raw + (footprint_estimate(req.radix) if hit is None else 0)
        self._evict(need, keep=req.key)
        if self._held() + need > self.hbm_budget and (self.running or self._held() > 0):
            return False
        if hit is None:
            plan, batchable = self.backend.build(req)
            nbytes = self.backend.plan_bytes(plan)
            self.stats["built"] += 1
            shared = nbytes <= self.cache_budget
            if shared:
                self.cache[req.key] = (plan, nbytes, batchable)
                self.cache_bytes += nbytes
            else:
                self.reserved += nbytes
        else:
            self.cache.move_to_end(req.key)
            self.stats["cache_hits"] += 1
            plan, nbytes, batchable = hit
            shared = True
        self.peak_bytes = max(self.peak_bytes, self._held())
        if not batchable:
            # a space the batched sweep cannot take runs alone
            pr, mins, info = self.backend.plain(plan, req)
            self._finish(req, pr, mins, info)
            if not shared:
                self._release(plan, nbytes)
            return True
        mbytes = self.backend.member_bytes(plan)
        self.reserved += mbytes
        self.peak_bytes = max(self.peak_bytes, self._held())
        self.backend.add(plan, req)
        if shared:
            self.in_use[req.key] = self.in_use.get(req.key, 0) + 1
        self.running[req.rid] = (req, req.key, plan, nbytes, shared, mbytes)
        return True

    def _release(self, plan, nbytes) -> None:
        self.reserved -= nbytes
        self.backend.release(plan)

    def _finish(self, req: Request, pr, mins, info) -> None:
        self.done.append(Done(req.rid, req.arrival, self.clock(), float(info["score"]), pr, mins, info))

    # -- main loop ----------------------------------------------------------
    def run(self, requests, start: float | None = None) -> list:
        """Serve `requests` (sorted by arrival, times relative to `start`)
        until all are done; returns the Done records."""
        paused = self.pause_gc and gc.isenabled()
        if paused:
            gc.disable()
        try:
            return self._loop(requests, start)
        finally:
            if paused:
                gc.enable()

    def _loop(self, requests, start) -> list:
        pending = list(requests)
        heapq.heapify(pending)
        t0 = self.clock() if start is None else start
        while pending or self.queue or self.running:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                self.queue.append(heapq.heappop(pending))
            still = []
            for req in self.queue:
                if not self._admit(_shift(req, t0)):
                    still.append(req)
            self.queue = still
            if self.running:
                self.backend.step()
                for tag, pr, mins, info in self.backend.collect():
                    req, key, plan, nbytes, shared, mbytes = self.running.pop(tag)
                    self.reserved -= mbytes
                    self._finish(req, pr, mins, info)
                    if shared:
                        self.in_use[key] -= 1
                    else:
                        self._release(plan, nbytes)
            elif pending and not self.queue:
                wait = pending[0].arrival - (self.clock() - t0)
                if wait > 0:
                    if self.pause_gc:
                        gc.collect(1)         # idle: young generations only
                        self.stats["gc_idle"] += 1
                        wait = pending[0].arrival - (self.clock() - t0)
                    if wait > 0:
                        self.sleep(min(wait, 0.001))
        return self.done


def _shift(req: Request, t0: float) -> Request:
    """The request with its arrival on the server's absolute clock."""
    if getattr(req, "_abs", False):
        return req
    r = Request(req.arrival + t0, req.rid, req.key, req.radix, req.fitness, req.neighbourhood,
                req.damping, req.p)
    r._abs = True
    return r


def serve_plain(backend, requests, clock: Callable[[], float] | None = None,
                start: float | None = None, sleep: Callable[[float], None] | None = None) -> list:
    """The one-at-a-time reference: FIFO, each analysis run alone with a
    fresh FFG build, in arrival order."""
    clock = clock or time.perf_counter
    sleep = sleep or time.sleep
    t0 = clock() if start is None else start
    done = []
    for req in sorted(requests):
        while True:
            wait = req.arrival - (clock() - t0)
            if wait <= 0:
                break
            sleep(min(wait, 0.001))
        plan, _ = backend.build(req)
        pr, mins, info = backend.plain(plan, req)
        backend.release(plan)
        done.append(Done(req.rid, req.arrival + t0, clock(), float(info["score"]), pr, mins, info))
    return done


def poisson_arrivals(rate: float, duration: float, seed: int = 5):
    """Arrival times of a Poisson stream (numpy PCG64, fixed seed)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return out
        out.append(t)


def latency_summary(done: list, since: float = 0.0) -> dict:
    import numpy as np
    t0 = min(d.arrival for d in done) if done else 0.0
    lat = np.array([d.latency for d in done if d.arrival - t0 >= since]) if done else np.zeros(0)
    if lat.size == 0:
        return {"n": 0}
    span = max(d.finish for d in done) - min(d.arrival for d in done)
    edges = sum(float(d.info.get("n_edges", 0)) * float(d.info.get("iterations", 0)) for d in done)
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "throughput_per_s": float(len(done) / span) if span > 0 else None,
            "gteps": float(edges / span / 1e9) if span > 0 else None}
