"""GPU: the continuous-batching server.  Every request's result equals the
same analysis run alone, whatever it shared the device with."""
import numpy as np
import pytest

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
    for r in reqs[:40]:
        plan = api.plan_create(ctx, r.radix, r.fitness, "hamming")
        pr, mins, info = api.execute(plan, r.damping, r.p, row_mapping=-1)
        assert np.array_equal(done[r.rid].pagerank.cpu().numpy(), pr.cpu().numpy())
        assert done[r.rid].score == info["score"]
        plan.close()
    summ = serve.latency_summary(list(done.values()))
    assert summ["p99_ms"] >= summ["p50_ms"] > 0
    backend.close()
    for cached in list(srv.cache.values()):
        cached[0].close()
    ctx.close()
