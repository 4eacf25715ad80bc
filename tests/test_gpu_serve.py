"""GPU: the continuous-batching server.  Every request's result equals the
same analysis run alone (batch members: with the batch's separate step;
requests that found the server idle: the lagged single-space path),
whatever it shared the device with, and matches the FP64 oracle (minima
exactly, ranks within 1e-5 in L1, C_p within 1e-5)."""
import collections
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2210_01465_amd import serve, synth

pytestmark = pytest.mark.gpu


def test_served_equals_alone():
    import torch
    from paper_2210_01465_amd import api
    ctx = api.Context(0)
    spaces = synth.batched()[::7] + [synth.mid()]
    fits = [torch.from_numpy(s.fitness_raw).cuda() for s in spaces]
    rng = np.random.default_rng(1)
    times = serve.poisson_arrivals(3000.0, 0.1, seed=1)
    reqs = []
    for rid, t in enumerate(times):
        j = int(rng.integers(len(spaces)))
        reqs.append(serve.Request(t, rid, (j, "hamming"), spaces[j].radix, fits[j], "hamming",
                                  float(rng.choice([0.8, 0.85, 0.9])), 0.05))
    print(f"[case] serve {len(reqs)} requests over {len(spaces)} spaces", flush=True)
    backend = serve.GpuBackend(ctx, sweeps_per_step=3)
    srv = serve.Server(backend, hbm_budget=8 << 30)
    done = {d.rid: d for d in srv.run(reqs)}
    assert sorted(done) == [r.rid for r in reqs]
    assert srv.stats["cache_hits"] > 0
    paths = collections.Counter(d.path for d in done.values())
    print(f"[case] paths {dict(paths)}", flush=True)
    assert paths["alone"] > 0 and paths["batch"] > 0
    picked = [r for r in reqs if done[r.rid].path == "batch"][:25] + \
        [r for r in reqs if done[r.rid].path == "alone"][:25]
    for r in picked:
        plan = api.plan_create(ctx, r.radix, r.fitness, "hamming")
        if done[r.rid].path == "batch":
            pr, mins, info = api.execute(plan, r.damping, r.p, row_mapping=-1, separate_step=True)
        else:
            pr, mins, info = api.execute(plan, r.damping, r.p)
        assert np.array_equal(done[r.rid].pagerank.cpu().numpy(), pr.cpu().numpy()), (r.rid, done[r.rid].path)
        assert np.array_equal(done[r.rid].minima.cpu().numpy(), mins.cpu().numpy())
        assert done[r.rid].score == info["score"]
        plan.close()
    summ = serve.latency_summary(list(done.values()))
    assert summ["p99_ms"] >= summ["p50_ms"] > 0
    backend.close()
    for cached in list(srv.cache.values()):
        cached[0].close()
    ctx.close()


@pytest.fixture(scope="module")
def large_reference():
    """The 1.5 M-node workload (10 parameters, 4 665 600 raw configurations)
    and its FP64 oracle analyses at d = 0.85 and 0.9, computed once."""
    s = synth.large()
    with ThreadPoolExecutor(2) as ex:
        refs = dict(zip((0.85, 0.9), ex.map(
            lambda d: oracle.analyze(s.radix, s.fitness_raw, oracle.HAMMING, d, 0.05, tol=1e-12), (0.85, 0.9))))
    return s, refs


def test_served_results_match_oracle(large_reference):
    """A Poisson stream mixing batched-workload spaces, the mid space and two
    requests for the 1.5 M-node space (as in the serving mix, where 2 % of
    requests are that space), damping drawn from {0.8, 0.85, 0.9}: every
    served result against the FP64 oracle."""
    import torch
    from paper_2210_01465_amd import api
    large, large_refs = large_reference
    ctx = api.Context(0)
    spaces = synth.batched()[::9] + [synth.mid()]
    fits = [torch.from_numpy(s.fitness_raw).cuda() for s in spaces]
    large_fit = torch.from_numpy(large.fitness_raw).cuda()
    rng = np.random.default_rng(7)
    times = serve.poisson_arrivals(2000.0, 0.06, seed=7)
    reqs = []
    for rid, t in enumerate(times):
        j = int(rng.integers(len(spaces)))
        reqs.append(serve.Request(t, rid, (j, "hamming"), spaces[j].radix, fits[j], "hamming",
                                  float(rng.choice([0.8, 0.85, 0.9])), 0.05))
    # the large space arrives twice, once early and once in the middle of the stream
    for k, (t, d) in enumerate(((times[2], 0.85), (times[len(times) // 2], 0.9))):
        reqs.append(serve.Request(t, len(times) + k, ("large", "hamming"), large.radix, large_fit,
                                  "hamming", d, 0.05))
    reqs.sort()
    # a space with 398 candidate slots per configuration (binned rows in the batch)
    wide = synth.Space("wide", (200, 3), rng.lognormal(0.0, 0.5, 600).astype(np.float32))
    wide_fit = torch.from_numpy(wide.fitness_raw).cuda()
    spaces.append(wide)
    for k, t in enumerate((times[5], times[-5])):
        reqs.append(serve.Request(t, len(times) + 2 + k, (len(spaces) - 1, "hamming"), wide.radix, wide_fit,
                                  "hamming", 0.85, 0.05))
    reqs.sort()
    print(f"[case] serve {len(reqs)} requests ({len(spaces)} spaces + 2 large) against the oracle, "
          f"FFG builds, graphs above 4 M edges and lone requests on the builder thread", flush=True)
    backend = serve.GpuBackend(ctx, sweeps_per_step=8, async_builds=True)
    srv = serve.Server(backend, hbm_budget=16 << 30, alone_edges=1 << 22, alone_on_builder=True,
                       switch_interval=1e-4)
    done = {d.rid: d for d in srv.run(reqs)}
    assert sorted(done) == sorted(r.rid for r in reqs)
    print(f"[case] paths {dict(collections.Counter(d.path for d in done.values()))}", flush=True)
    assert all(done[r.rid].path == "builder" for r in reqs if r.key[0] == "large")
    assert srv.stats["built"] == len({r.key for r in reqs})
    keys = sorted({(r.key[0], r.damping) for r in reqs if r.key[0] != "large"}, key=str)

    def ref(kd):
        j, d = kd
        return oracle.analyze(spaces[j].radix, spaces[j].fitness_raw, oracle.HAMMING, d, 0.05, tol=1e-12)
    with ThreadPoolExecutor(8) as ex:
        refs = dict(zip(keys, ex.map(ref, keys)))
    refs.update({("large", d): a for d, a in large_refs.items()})
    worst = 0.0
    for r in reqs:
        a = refs[(r.key[0], r.damping)]
        got = done[r.rid]
        assert got.info["status"] == 0, r.rid
        assert np.array_equal(got.minima.cpu().numpy(), a.graph.minima), (r.rid, r.key)
        l1 = float(np.abs(got.pagerank.cpu().numpy() - a.pagerank).sum())
        assert l1 <= 1e-5, (r.rid, r.key, l1)
        assert abs(got.score - a.score) <= 1e-5, (r.rid, r.key, got.score, a.score)
        worst = max(worst, l1)
    print(f"[case] worst served L1 vs oracle {worst:.3e}", flush=True)
    srv.close()
    backend.close()
    ctx.close()
