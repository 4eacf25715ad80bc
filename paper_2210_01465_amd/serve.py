"""Continuous-batching server for landscape analyses.

Requests (a search space, its fitness on the GPU, a neighbourhood, d and p)
arrive over time.  The server

* admits a request once its estimated device footprint fits under an HBM
  budget (default: the device's free memory at start-up minus a reserve),
  queueing it otherwise;
* keeps built fitness flow graphs in a device-resident LRU cache keyed by the
  request's content key, so a repeated space with another d or p only reruns
  PageRank;
* builds the FFG of a cache miss off the serving loop when the backend can
  (``GpuBackend(async_builds=True)``: a builder thread with its own engine
  context on a second stream, so the build's kernels overlap the running
  batch and no step waits for it); requests for a space whose build is in
  flight wait for that build instead of starting another;
* adds admitted requests to one running batch (fl_batch_*): members join and
  leave between steps of a few sweeps, so short analyses are not held behind
  long ones;
* runs a request alone, at once, on the single-space path (lagged step, no
  batch bookkeeping) when it finds the server idle: no batch member running
  and no other request waiting to start.  Under light load most requests
  take this path and see the single-space latency; as soon as requests
  overlap they batch.  Optionally (``alone_edges``), analyses of graphs above
  that many edges run alone on the builder's stream beside the batch, so
  short requests never wait behind them, and (``alone_on_builder``) a
  request that cannot run alone at once runs alone on the builder if it is
  idle;
* records, per request, the latency from arrival to a host-visible result;
* keeps Python's cyclic garbage collector from running inside the loop (a
  full collection over the live request and tensor objects stalls the loop
  for tens of milliseconds): automatic collection is paused while ``run``
  serves and the young generations are collected when the loop idles.

The GPU work goes through a backend object (``build``, ``plan_bytes``,
``member_bytes``, ``add``, ``step``, ``collect``, ``release``, plus ``plain``
for the one-at-a-time reference path; optionally ``alone`` (the idle fast
path) and ``edges``; a backend with ``async_builds`` set also has
``submit_build`` / ``submit_plain`` / ``poll``), so the scheduling logic can
be exercised with any backend.
"""
from __future__ import annotations

import collections
import gc
import heapq
import queue
import sys
import threading
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
    path: str = "batch"     # batch | alone (idle fast path) | builder (alone on its stream) | plain

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


class _Builder:
    """A thread that owns a second engine context on its own stream (default
    priority) and runs FFG builds, lone analyses of spaces the batch cannot
    take, and plan releases for that context, one job at a time.  The engine
    calls release the interpreter lock, so its kernels run while the serving
    loop steps the batch on the first context's stream.  Fitness tensors
    handed to it must have no pending writes.  ``lock`` is held while a job
    runs; the serving thread takes it to use the builder's context itself."""

    def __init__(self, api, device: int):
        import torch
        self.api = api
        self.device = device
        self.stream = torch.cuda.Stream(device=device)
        self.ctx = api.Context(device, self.stream)
        self.jobs: "queue.Queue" = queue.Queue()
        self.done: "queue.Queue" = queue.Queue()
        self.lock = threading.Lock()
        self.thread = threading.Thread(target=self._run, name="ffg-builder", daemon=True)
        self.thread.start()

    def _run(self):
        import torch
        torch.cuda.set_device(self.device)
        with torch.cuda.stream(self.stream):
            while True:
                job = self.jobs.get()
                if job is None:
                    return
                kind, a, b = job
                try:
                    self.lock.acquire()
                    if kind == "build":
                        plan = self.api.plan_create(self.ctx, a.radix, a.fitness, a.neighbourhood)
                        self.done.put(("build", a, (plan, _batchable(plan)), None))
                    elif kind == "plain":
                        self.done.put(("plain", b, self.api.execute(a, b.damping, b.p), None))
                    else:
                        a.close()
                except Exception as e:          # handed to the serving loop, which raises it
                    self.done.put((kind, a if kind == "build" else b, None, e))
                finally:
                    self.lock.release()

    def close(self):
        self.jobs.put(None)
        self.thread.join()
        self.ctx.close()


def _batchable(plan) -> bool:
    """Whether a batch can take the plan: a space without slot records has
    its rows binned when it is built (binned sweep); one with them needs the
    slot sweep's buffer loads (4 n_raw < 2^31)."""
    words = int(plan.sizes.get("mask_words", 0))
    return words == 0 or 4 * plan.sizes["n_raw"] < 2 ** 31


class GpuBackend:
    """The engine through the Python binding (one context, one batch; with
    async_builds, a builder thread with a second context for cache misses)."""

    def __init__(self, ctx=None, sweeps_per_step: int = 16, async_builds: bool = False):
        from . import api
        self.api = api
        self.ctx = ctx or api.Context(0)
        self.batch = api.Batch(self.ctx)
        self.sweeps = sweeps_per_step
        self.async_builds = bool(async_builds)
        self.builder = _Builder(api, self.ctx.device) if async_builds else None

    def build(self, req: Request):
        plan = self.api.plan_create(self.ctx, req.radix, req.fitness, req.neighbourhood)
        return plan, _batchable(plan)

    def submit_build(self, req: Request) -> None:
        self.builder.jobs.put(("build", req, None))

    def submit_plain(self, plan, req: Request) -> None:
        self.builder.jobs.put(("plain", plan, req))

    def poll(self) -> list:
        """Finished builder jobs: ("build", req, (plan, batchable)) and
        ("plain", req, (pagerank, minima, info)); a job that failed raises."""
        out = []
        while True:
            try:
                kind, req, res, err = self.builder.done.get_nowait()
            except queue.Empty:
                return out
            if err is not None:
                raise err
            out.append((kind, req, res))

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

    def alone(self, plan, req: Request):
        """Run one request alone at once on the calling thread (the
        single-space path), or return None when the plan's context is busy:
        a plan built by the builder runs on the builder's context and stream,
        which the builder must not be using."""
        b = self.builder
        if b is None or plan.ctx is not b.ctx:
            return self.plain(plan, req)
        if not b.lock.acquire(blocking=False):
            return None
        try:
            import torch
            with torch.cuda.stream(b.stream):
                return self.plain(plan, req)
        finally:
            b.lock.release()

    def edges(self, plan) -> int:
        return int(plan.sizes["n_edges"])

    def release(self, plan) -> None:
        if self.builder is not None and plan.ctx is self.builder.ctx:
            self.builder.jobs.put(("release", plan, None))   # its context belongs to the builder thread
        else:
            plan.close()

    def sync(self) -> None:
        import torch
        torch.cuda.synchronize()

    def close(self) -> None:
        """Release the batch and the builder (after the plans it built)."""
        self.batch.close()
        if self.builder is not None:
            self.builder.close()
            self.builder = None


class Server:
    """Continuous-batching scheduler (see the module docstring).

    Plans are held in the LRU cache (shared by any number of requests) or,
    when larger than the cache budget, owned by the requests of their key and
    released when the last of them finishes.  Memory accounting: every
    admitted request reserves 16 n_raw bytes for its own iterates until it
    joins (then its member bytes), and a build in flight reserves the
    estimated footprint of its FFG until the plan's own size is known.

    alone_when_idle: use the backend's ``alone`` (if it has one) for a
    request that finds the server idle.  alone_edges: with an async backend,
    analyses of plans above this many edges run alone on the builder instead
    of joining the batch (None: never).  alone_on_builder: with an async
    backend, a request that cannot run alone at once runs alone on the
    builder when the builder is idle, instead of joining the batch.
    switch_interval: the interpreter's thread switch interval while ``run``
    serves (None: unchanged); a short one lets the builder thread take the
    interpreter lock soon after its job is queued."""

    def __init__(self, backend, hbm_budget: int, cache_budget: int | None = None,
                 clock: Callable[[], float] | None = None,
                 sleep: Callable[[float], None] | None = None, pause_gc: bool = True,
                 alone_when_idle: bool = True, alone_edges: int | None = None,
                 alone_on_builder: bool = False, switch_interval: float | None = None):
        self.backend = backend
        self.async_builds = bool(getattr(backend, "async_builds", False))
        self.alone_when_idle = bool(alone_when_idle) and hasattr(backend, "alone")
        self.alone_edges = alone_edges if self.async_builds else None
        self.alone_on_builder = bool(alone_on_builder) and self.async_builds
        self.switch_interval = switch_interval
        self.pause_gc = pause_gc
        self.hbm_budget = int(hbm_budget)
        self.cache_budget = int(cache_budget if cache_budget is not None else hbm_budget // 2)
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.cache: "collections.OrderedDict[Hashable, tuple]" = collections.OrderedDict()
        self.cache_bytes = 0
        self.in_use: dict = {}            # key -> requests using the cached plan
        self.owned: dict = {}             # key -> [plan, nbytes, batchable, users] (plans above the cache budget)
        self.reserved = 0                 # bytes of owned plans, members and admitted requests' iterates
        self.building: dict = {}          # key -> requests waiting for the build in flight
        self.building_bytes: dict = {}    # key -> estimated footprint reserved for that build
        self.plain_inflight = 0           # lone analyses running on the builder
        self.peak_bytes = 0
        self.queue: list = []             # admitted order: waiting requests
        self.running: dict = {}           # rid -> (req, key, member bytes)
        self.done: list = []
        self.stats = collections.Counter()

    # -- memory accounting -------------------------------------------------
    def _held(self) -> int:
        return self.cache_bytes + self.reserved + sum(self.building_bytes.values())

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

    @staticmethod
    def _iterate_estimate(req: Request) -> int:
        n_raw = 1
        for r in req.radix:
            n_raw *= int(r)
        return 16 * n_raw

    def _admit(self, req: Request, alone_ok: bool = False) -> bool:
        """Reserve memory for the request and start it: join the batch at
        once on a cached (or owned) plan, wait for a build of its space that
        is in flight, or start that build.  False leaves it queued.
        alone_ok: no other request is starting with it."""
        key = req.key
        hit = self.cache.get(key)
        known = hit is not None or key in self.owned or key in self.building
        it_bytes = self._iterate_estimate(req)
        build_bytes = 0 if known else footprint_estimate(req.radix)
        need = it_bytes + build_bytes
        self._evict(need, keep=key)
        if self._held() + need > self.hbm_budget and (self.running or self._held() > 0):
            return False
        self.reserved += it_bytes
        self.peak_bytes = max(self.peak_bytes, self._held() + build_bytes)
        if hit is not None:
            self.cache.move_to_end(key)
            self.stats["cache_hits"] += 1
            self._start(req, key, hit[0], hit[2], it_bytes, alone_ok)
        elif key in self.owned:
            self.stats["cache_hits"] += 1
            self._start(req, key, self.owned[key][0], self.owned[key][2], it_bytes, alone_ok)
        elif key in self.building:
            self.stats["build_waits"] += 1
            self.building[key].append(req)
        elif self.async_builds:
            self.stats["built"] += 1
            self.building[key] = [req]
            self.building_bytes[key] = build_bytes
            self.backend.submit_build(req)
        else:
            self.stats["built"] += 1
            plan, batchable = self.backend.build(req)
            self._store(key, plan, batchable)
            self._start(req, key, plan, batchable, it_bytes, alone_ok)
        self.peak_bytes = max(self.peak_bytes, self._held())
        return True

    def _store(self, key, plan, batchable) -> None:
        """A plan just built: into the cache if it fits the cache budget, else
        owned by the requests of its key."""
        nbytes = self.backend.plan_bytes(plan)
        if nbytes <= self.cache_budget:
            self.cache[key] = (plan, nbytes, batchable)
            self.cache_bytes += nbytes
        else:
            self.owned[key] = [plan, nbytes, batchable, 0]
            self.reserved += nbytes

    def _use(self, key, delta: int) -> None:
        if key in self.owned:
            o = self.owned[key]
            o[3] += delta
            if o[3] == 0:
                del self.owned[key]
                self.reserved -= o[1]
                self.backend.release(o[0])
        else:
            self.in_use[key] = self.in_use.get(key, 0) + delta

    def _start(self, req: Request, key, plan, batchable, it_bytes: int, alone_ok: bool = False) -> None:
        """Run an admitted request on its plan: alone on the builder when the
        batched sweep cannot take the space (or the graph is above
        alone_edges); alone at once when it finds the server idle (alone_ok
        and no batch member running); alone on the idle builder with
        alone_on_builder; else as a batch member."""
        self._use(key, +1)
        if batchable and self.alone_edges is not None and self.backend.edges(plan) > self.alone_edges:
            batchable = False
        if not batchable:
            if self.async_builds:
                self.plain_inflight += 1
                self.running[req.rid] = (req, key, it_bytes)
                self.backend.submit_plain(plan, req)
            else:
                pr, mins, info = self.backend.plain(plan, req)
                self.reserved -= it_bytes
                self._finish(req, pr, mins, info, "plain")
                self._use(key, -1)
            return
        if alone_ok and self.alone_when_idle and len(self.running) == self.plain_inflight:
            res = self.backend.alone(plan, req)
            if res is not None:
                self.stats["alone"] += 1
                self.reserved -= it_bytes
                self._finish(req, *res, "alone")
                self._use(key, -1)
                return
        if self.alone_on_builder and self.plain_inflight == 0 and not self.building:
            self.stats["alone_builder"] += 1
            self.plain_inflight += 1
            self.running[req.rid] = (req, key, it_bytes)
            self.backend.submit_plain(plan, req)
            return
        mbytes = self.backend.member_bytes(plan)
        self.reserved += mbytes - it_bytes
        self.peak_bytes = max(self.peak_bytes, self._held())
        self.backend.add(plan, req)
        self.running[req.rid] = (req, key, mbytes)

    def _end(self, rid, pr, mins, info, path: str = "batch") -> None:
        req, key, nbytes = self.running.pop(rid)
        self.reserved -= nbytes
        self._finish(req, pr, mins, info, path)
        self._use(key, -1)

    def _finish(self, req: Request, pr, mins, info, path: str) -> None:
        self.done.append(Done(req.rid, req.arrival, self.clock(), float(info["score"]), pr, mins, info, path))

    def _poll_builder(self) -> None:
        for kind, req, res in self.backend.poll():
            if kind == "build":
                plan, batchable = res
                key = req.key
                waiting = self.building.pop(key)
                self.building_bytes.pop(key)
                self._store(key, plan, batchable)
                lone = len(waiting) == 1 and not self.queue
                for r in waiting:
                    self._start(r, key, plan, batchable, self._iterate_estimate(r), lone)
                self.peak_bytes = max(self.peak_bytes, self._held())
            else:
                self.plain_inflight -= 1
                self._end(req.rid, *res, "builder")

    # -- main loop ----------------------------------------------------------
    def run(self, requests, start: float | None = None) -> list:
        """Serve `requests` (sorted by arrival, times relative to `start`)
        until all are done; returns the Done records."""
        paused = self.pause_gc and gc.isenabled()
        if paused:
            gc.disable()
        interval = sys.getswitchinterval()
        if self.switch_interval is not None:
            sys.setswitchinterval(self.switch_interval)
        try:
            return self._loop(requests, start)
        finally:
            sys.setswitchinterval(interval)
            if paused:
                gc.enable()

    def _loop(self, requests, start) -> list:
        pending = list(requests)
        heapq.heapify(pending)
        t0 = self.clock() if start is None else start
        while pending or self.queue or self.running or self.building:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                self.queue.append(heapq.heappop(pending))
            if self.async_builds:
                self._poll_builder()
            still = []
            lone = len(self.queue) == 1
            for req in self.queue:
                if not self._admit(_shift(req, t0), lone):
                    still.append(req)
            self.queue = still
            members = len(self.running) - self.plain_inflight
            if members > 0:
                self.backend.step()
                for tag, pr, mins, info in self.backend.collect():
                    self._end(tag, pr, mins, info)
            elif self.building or self.plain_inflight:
                self.sleep(5e-5)              # only builder work in flight
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

    def close(self) -> None:
        """Release every cached plan (the server must be idle)."""
        for plan, _, _ in self.cache.values():
            self.backend.release(plan)
        self.cache.clear()
        self.cache_bytes = 0


def _shift(req: Request, t0: float) -> Request:
    """The request with its arrival on the server's absolute clock."""
    if getattr(req, "_abs", False):
        return req
    r = Request(req.arrival + t0, req.rid, req.key, req.radix, req.fitness, req.neighbourhood,
                req.damping, req.p)
    r._abs = True
    return r


def serve_plain(backend, requests, clock: Callable[[], float] | None = None,
                start: float | None = None, sleep: Callable[[float], None] | None = None,
                cache_budget: int = 0) -> list:
    """The one-at-a-time reference: FIFO, each analysis run alone in arrival
    order.  With cache_budget > 0 it keeps the same kind of content-keyed LRU
    plan cache as the server (plans up to that many bytes in total), so a
    repeated space reruns only PageRank; with 0 every request builds its FFG."""
    clock = clock or time.perf_counter
    sleep = sleep or time.sleep
    t0 = clock() if start is None else start
    cache: "collections.OrderedDict[Hashable, tuple]" = collections.OrderedDict()
    held = 0
    done = []
    for req in sorted(requests):
        while True:
            wait = req.arrival - (clock() - t0)
            if wait <= 0:
                break
            sleep(min(wait, 0.001))
        hit = cache.get(req.key)
        if hit is not None:
            cache.move_to_end(req.key)
            plan = hit[0]
        else:
            plan, _ = backend.build(req)
            nbytes = backend.plan_bytes(plan)
            if nbytes <= cache_budget:
                while cache and held + nbytes > cache_budget:
                    old, ob = cache.popitem(last=False)[1]
                    held -= ob
                    backend.release(old)
                cache[req.key] = (plan, nbytes)
                held += nbytes
        pr, mins, info = backend.plain(plan, req)
        if req.key not in cache:
            backend.release(plan)
        done.append(Done(req.rid, req.arrival + t0, clock(), float(info["score"]), pr, mins, info, "plain"))
    for plan, _ in cache.values():
        backend.release(plan)
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
    # over the measured requests alone: from the first measured arrival to the last of their results
    meas = [d for d in done if d.arrival - t0 >= since]
    mspan = max(d.finish for d in meas) - min(d.arrival for d in meas)
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3),
            "throughput_per_s": float(len(done) / span) if span > 0 else None,
            "measured_throughput_per_s": float(len(meas) / mspan) if mspan > 0 else None,
            "gteps": float(edges / span / 1e9) if span > 0 else None}
