"""Serving scheduler on the CPU: a fake backend (built on the oracle) stands
in for the GPU engine, with a virtual clock, so admission, the FFG cache and
continuous batching are tested without a device."""
import gc

import numpy as np
import pytest

import oracle
from paper_2210_01465_amd import serve, synth


class FakeBackend:
    """Members finish after as many steps as their oracle iteration count
    needs; every build/step advances a virtual clock."""

    def __init__(self, sweeps_per_step=4, step_cost=1e-4, build_cost=2e-4):
        self.now = 0.0
        self.sweeps = sweeps_per_step
        self.step_cost, self.build_cost = step_cost, build_cost
        self.members = {}
        self.built = []
        self.live_plans = 0
        self.added_while_running = 0
        self.max_on_one_plan = 0                  # members sharing one FFG at once
        self.gc_during_step = set()
        self.n_builds = 0

    def clock(self):
        return self.now

    def sleep(self, dt):
        self.now += dt

    def build(self, req):
        self.now += self.build_cost
        self.n_builds += 1
        self.live_plans += 1
        g = oracle.build_graph(req.radix, req.fitness, {"hamming": 0, "adjacent": 1}[req.neighbourhood])
        self.built.append(g)
        return g, True

    def plan_bytes(self, g):
        return 64 * g.n_raw

    def member_bytes(self, g):
        return 16 * g.n_raw

    def add(self, g, req):
        if self.members:
            self.added_while_running += 1
        r, it, _ = g.pagerank(req.damping, 2e-7)
        sc = g.score(r, req.p)[0]
        self.members[req.rid] = [it, r, g.minima, {"score": sc, "iterations": it, "status": 0}, g]
        self.max_on_one_plan = max(self.max_on_one_plan,
                                   sum(1 for m in self.members.values() if m[4] is g))

    def step(self):
        self.gc_during_step.add(gc.isenabled())
        self.now += self.step_cost
        for m in self.members.values():
            m[0] -= self.sweeps
        return sum(1 for m in self.members.values() if m[0] > 0)

    def collect(self):
        out = [(rid, m[1], m[2], m[3]) for rid, m in self.members.items() if m[0] <= 0]
        assert all(any(m[4] is b for b in self.built) for m in self.members.values())   # no member outlives its plan
        for rid, *_ in out:
            del self.members[rid]
        return out

    def plain(self, g, req):
        r, it, _ = g.pagerank(req.damping, 2e-7)
        self.now += self.step_cost * (it // self.sweeps + 1)
        return r, g.minima, {"score": g.score(r, req.p)[0], "iterations": it, "status": 0}

    def release(self, g):
        self.live_plans -= 1
        self.built = [b for b in self.built if b is not g]


def make_requests(n, seed=0, rate=2000.0):
    spaces = [synth.tiny(s) for s in range(3)] + [synth.fuzz_space(j, max_params=4, max_radix=6) for j in range(5)]
    spaces = [s for s in spaces if s.n_valid > 0]
    rng = np.random.default_rng(seed)
    times = serve.poisson_arrivals(rate, n / rate, seed=seed)
    reqs = []
    for rid, t in enumerate(times[:n]):
        j = int(rng.integers(len(spaces)))
        s = spaces[j]
        reqs.append(serve.Request(t, rid, (j, "hamming"), s.radix, s.fitness_raw, "hamming",
                                  float(rng.choice([0.8, 0.85, 0.9])), 0.05))
    return reqs


def test_every_request_matches_its_plain_result():
    reqs = make_requests(60)
    fb = FakeBackend()
    srv = serve.Server(fb, hbm_budget=1 << 30, clock=fb.clock, sleep=fb.sleep)
    done = {d.rid: d for d in srv.run(reqs)}
    assert sorted(done) == [r.rid for r in reqs]
    for r in reqs:
        g = oracle.build_graph(r.radix, r.fitness)
        rr, _, _ = g.pagerank(r.damping, 2e-7)
        assert done[r.rid].score == g.score(rr, r.p)[0]
        assert done[r.rid].latency >= 0
    assert fb.added_while_running > 0          # members joined a running batch
    assert srv.stats["cache_hits"] > 0         # repeated spaces reuse their FFG
    assert srv.stats["built"] <= 8
    assert fb.max_on_one_plan >= 2             # one cached FFG ran for several requests at once


def test_admission_respects_the_budget():
    reqs = make_requests(40, seed=3, rate=50000.0)
    fb = FakeBackend()
    budget = 3 * (64 + 16) * 160 + (1 << 20) * 3   # room for about three tiny spaces
    srv = serve.Server(fb, hbm_budget=budget, cache_budget=0, clock=fb.clock, sleep=fb.sleep)
    done = srv.run(reqs)
    assert len(done) == len(reqs)
    assert srv.peak_bytes <= budget
    assert fb.live_plans == 0                   # nothing cached (cache budget 0): all released


def test_plain_path_and_summary():
    reqs = make_requests(20, seed=4)
    fb = FakeBackend()
    done = serve.serve_plain(fb, reqs, clock=fb.clock, sleep=fb.sleep)
    assert [d.rid for d in done] == sorted(r.rid for r in reqs)
    summ = serve.latency_summary(done)
    assert summ["n"] == len(reqs) and summ["p99_ms"] >= summ["p50_ms"] >= 0


def test_poisson_arrivals_are_seeded():
    a = serve.poisson_arrivals(1000.0, 0.5, seed=5)
    b = serve.poisson_arrivals(1000.0, 0.5, seed=5)
    assert a == b and 400 < len(a) < 600 and all(x < y for x, y in zip(a, a[1:]))


@pytest.mark.parametrize("pause", [True, False])
def test_collector_paused_while_serving(pause):
    """Automatic garbage collection is off inside the loop (collected only
    when idle) and back on afterwards, unless the server is told otherwise."""
    reqs = make_requests(30, seed=6, rate=500.0)
    fb = FakeBackend()
    srv = serve.Server(fb, hbm_budget=1 << 30, clock=fb.clock, sleep=fb.sleep, pause_gc=pause)
    assert gc.isenabled()
    done = srv.run(reqs)
    assert gc.isenabled() and len(done) == len(reqs)
    assert fb.gc_during_step == {not pause}
    assert (srv.stats["gc_idle"] > 0) == pause


class FakeAsyncBackend(FakeBackend):
    """Builds (and lone analyses of spaces marked unbatchable) run off the
    loop: each completes build_cost (or its step cost) of virtual time after
    it was submitted, while the loop keeps stepping the batch."""
    async_builds = True

    def __init__(self, unbatchable=(), **kw):
        super().__init__(**kw)
        self.jobs = []                     # (ready time, kind, req, payload)
        self.unbatchable = set(unbatchable)
        self.steps_during_builds = 0

    def submit_build(self, req):
        g = oracle.build_graph(req.radix, req.fitness, {"hamming": 0, "adjacent": 1}[req.neighbourhood])
        self.built.append(g)
        self.live_plans += 1
        self.jobs.append((self.now + self.build_cost, "build", req, (g, req.key[0] not in self.unbatchable)))

    def submit_plain(self, g, req):
        r, it, _ = g.pagerank(req.damping, 2e-7)
        res = (r, g.minima, {"score": g.score(r, req.p)[0], "iterations": it, "status": 0})
        self.jobs.append((self.now + self.step_cost * (it // self.sweeps + 1), "plain", req, res))

    def poll(self):
        ready = [j for j in self.jobs if j[0] <= self.now]
        self.jobs = [j for j in self.jobs if j[0] > self.now]
        return [(kind, req, res) for _, kind, req, res in ready]

    def step(self):
        if any(j[1] == "build" for j in self.jobs):
            self.steps_during_builds += 1
        return super().step()


class FakeIdleBackend(FakeBackend):
    """With the idle fast path: ``alone`` runs the request at once."""

    def __init__(self, **kw):
        super().__init__(**kw)
        self.n_alone = 0

    def alone(self, g, req):
        assert not self.members                   # only when no batch member runs
        self.n_alone += 1
        return self.plain(g, req)


class FakeAsyncIdleBackend(FakeAsyncBackend):
    """Async builds plus the fast path, which (as with the real builder's
    lock) is refused while a builder job is in flight."""

    def alone(self, g, req):
        if self.jobs:
            return None
        return self.plain(g, req)

    def edges(self, g):
        return g.E


def _check_against_plain(reqs, done):
    assert sorted(done) == sorted(r.rid for r in reqs)
    for r in reqs:
        g = oracle.build_graph(r.radix, r.fitness)
        rr, _, _ = g.pagerank(r.damping, 2e-7)
        assert done[r.rid].score == g.score(rr, r.p)[0]


def test_async_builds_overlap_the_batch_and_are_shared():
    """Cache misses build off the loop: the batch keeps stepping while builds
    are in flight, requests for a space being built wait for that one build,
    and every result equals its plain result."""
    reqs = make_requests(80, seed=7, rate=20000.0)
    fb = FakeAsyncBackend(build_cost=5e-4)
    srv = serve.Server(fb, hbm_budget=1 << 30, clock=fb.clock, sleep=fb.sleep)
    done = {d.rid: d for d in srv.run(reqs)}
    _check_against_plain(reqs, done)
    keys = {r.key for r in reqs}
    assert srv.stats["built"] == len(keys)          # one build per distinct space
    assert srv.stats["build_waits"] > 0             # later requests joined a build in flight
    assert fb.steps_during_builds > 0               # the batch ran while builds were in flight
    assert not srv.building and not srv.running
    srv.close()
    assert fb.live_plans == 0


def test_async_unbatchable_spaces_and_budget():
    """Spaces the batch cannot take run alone on the builder; with no cache
    every plan is released once its requests finish, and the budget holds."""
    reqs = make_requests(50, seed=8, rate=50000.0)
    fb = FakeAsyncBackend(unbatchable={0, 2}, build_cost=3e-4)
    budget = 4 * (64 + 16) * 160 + (1 << 20) * 4
    srv = serve.Server(fb, hbm_budget=budget, cache_budget=0, clock=fb.clock, sleep=fb.sleep)
    done = {d.rid: d for d in srv.run(reqs)}
    _check_against_plain(reqs, done)
    assert srv.peak_bytes <= budget
    assert fb.live_plans == 0 and srv.reserved == 0


def test_plain_path_with_the_same_cache():
    """The one-at-a-time path with a plan cache builds each distinct space
    once; without one it builds per request.  Results are the same."""
    reqs = make_requests(40, seed=9)
    fb = FakeBackend()
    cached = {d.rid: d for d in serve.serve_plain(fb, reqs, clock=fb.clock, sleep=fb.sleep, cache_budget=1 << 30)}
    assert fb.n_builds == len({r.key for r in reqs}) and fb.live_plans == 0
    fb2 = FakeBackend()
    fresh = {d.rid: d for d in serve.serve_plain(fb2, reqs, clock=fb2.clock, sleep=fb2.sleep)}
    assert fb2.n_builds == len(reqs) and fb2.live_plans == 0
    assert {r.rid: cached[r.rid].score for r in reqs} == {r.rid: fresh[r.rid].score for r in reqs}


def test_idle_requests_run_alone_and_bursts_batch():
    """A request that finds the server idle runs alone at once; requests
    that overlap join the batch.  Every result equals its plain result."""
    light = make_requests(40, seed=11, rate=100.0)
    fb = FakeIdleBackend()
    srv = serve.Server(fb, hbm_budget=1 << 30, clock=fb.clock, sleep=fb.sleep)
    done = {d.rid: d for d in srv.run(light)}
    _check_against_plain(light, done)
    assert srv.stats["alone"] == fb.n_alone == sum(d.path == "alone" for d in done.values())
    assert srv.stats["alone"] >= 30 and srv.reserved == 0
    burst = make_requests(60, seed=12, rate=50000.0)
    fb = FakeIdleBackend()
    srv = serve.Server(fb, hbm_budget=1 << 30, clock=fb.clock, sleep=fb.sleep)
    done = {d.rid: d for d in srv.run(burst)}
    _check_against_plain(burst, done)
    assert fb.added_while_running > 0 and sum(d.path == "batch" for d in done.values()) > 30
    assert srv.reserved == 0
    fb = FakeIdleBackend()
    srv = serve.Server(fb, hbm_budget=1 << 30, clock=fb.clock, sleep=fb.sleep, alone_when_idle=False)
    done = srv.run(light)
    assert fb.n_alone == 0 and {d.path for d in done} == {"batch"}


def test_long_graphs_run_on_the_builder():
    """With alone_edges, graphs above that many edges run alone on the
    builder (beside the batch); the fast path waits for an idle builder."""
    reqs = make_requests(60, seed=13, rate=5000.0)
    fb = FakeAsyncIdleBackend(build_cost=3e-4)
    graphs = {r.key: oracle.build_graph(r.radix, r.fitness) for r in reqs}
    cut = int(np.median([g.E for g in graphs.values()]))
    srv = serve.Server(fb, hbm_budget=1 << 30, clock=fb.clock, sleep=fb.sleep, alone_edges=cut)
    done = {d.rid: d for d in srv.run(reqs)}
    _check_against_plain(reqs, done)
    for r in reqs:
        long = graphs[r.key].E > cut
        assert (done[r.rid].path == "builder") == long, (r.rid, done[r.rid].path)
    assert any(d.path == "builder" for d in done.values())
    assert any(d.path == "batch" for d in done.values())
    assert not srv.running and srv.plain_inflight == 0 and srv.reserved == 0
    srv.close()
    assert fb.live_plans == 0


def test_idle_builder_takes_lone_requests():
    """With alone_on_builder, a request that cannot run alone at once (a
    batch is running) runs alone on the builder when it is idle; the switch
    interval is restored after the run."""
    import sys
    reqs = make_requests(60, seed=14, rate=8000.0)
    fb = FakeAsyncIdleBackend(build_cost=1e-4)
    before = sys.getswitchinterval()
    srv = serve.Server(fb, hbm_budget=1 << 30, clock=fb.clock, sleep=fb.sleep, alone_on_builder=True,
                       switch_interval=1e-4)
    done = {d.rid: d for d in srv.run(reqs)}
    assert sys.getswitchinterval() == before
    _check_against_plain(reqs, done)
    paths = {d.path for d in done.values()}
    assert "builder" in paths and srv.stats["alone_builder"] > 0
    assert not srv.running and srv.plain_inflight == 0 and srv.reserved == 0
    srv.close()
    assert fb.live_plans == 0
