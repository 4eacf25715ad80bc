"""GPU: the sweep-layout autotuner (fl_tune) and its tuning cache.

The tuner times every layout a plan allows and caches the fastest per shape
class; the automatic mapping must then pick it, and the analysis must still
match the FP64 oracle (layout changes only the summation order).
"""
import numpy as np
import pytest

import oracle
from paper_2210_01465_amd import synth

pytestmark = pytest.mark.gpu

LAYOUTS = (-1, 1, 2, 4, 8, 16, 32, 64, -2)


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def api_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2210_01465_amd import api
    return api


@pytest.mark.parametrize("nb", ["hamming", "adjacent"])
def test_tune_then_auto_uses_choice(api_mod, nb):
    import torch
    api = api_mod
    space = synth.mid()
    say(f"tune mid nb={nb}")
    ctx = api.Context(0)          # own context: the tuning cache is per context
    try:
        fit = torch.from_numpy(space.fitness_raw).cuda()
        plan = api.plan_create(ctx, space.radix, fit, nb)
        res = api.tune(plan, sweeps=3)
        assert res["best"] in LAYOUTS
        assert set(res["us_per_sweep"]) == set(LAYOUTS)   # mid fits the slot records
        assert all(t > 0 for t in res["us_per_sweep"].values())
        assert res["us_per_sweep"][res["best"]] == min(res["us_per_sweep"].values())
        pr, mins, info = api.execute(plan, 0.85, 0.05)
        torch.cuda.synchronize()
        assert info["row_mapping"] == res["best"]
        o = oracle.analyze(space.radix, space.fitness_raw,
                           oracle.HAMMING if nb == "hamming" else oracle.ADJACENT, 0.85, 0.05)
        assert np.array_equal(mins.cpu().numpy(), o.graph.minima)
        assert float(np.abs(pr.cpu().numpy() - o.pagerank).sum()) <= 1e-5
        assert abs(info["score"] - o.score) <= 1e-5
        # an explicit layout still overrides the cache
        _, _, info2 = api.execute(plan, 0.85, 0.05, row_mapping=8)
        assert info2["row_mapping"] == 8
        plan.close()
    finally:
        ctx.close()


def test_tune_without_slot_records(api_mod):
    """A space with more than 256 candidate slots has only the CSR layouts."""
    import torch
    api = api_mod
    rng = np.random.default_rng(11)
    radix = (200, 3)
    f = rng.lognormal(0.0, 1.0, size=600).astype(np.float32)
    say("tune radix=(200,3) hamming")
    ctx = api.Context(0)
    try:
        plan = api.plan_create(ctx, radix, torch.from_numpy(f).cuda(), "hamming")
        assert plan.sizes["mask_words"] == 0
        res = api.tune(plan, sweeps=2)
        assert -1 not in res["us_per_sweep"] and res["best"] in LAYOUTS[1:]
        pr, mins, info = api.execute(plan, 0.85, 0.05)
        assert info["row_mapping"] == res["best"]
        o = oracle.analyze(radix, f, oracle.HAMMING, 0.85, 0.05)
        assert float(np.abs(pr.cpu().numpy() - o.pagerank).sum()) <= 1e-5
        plan.close()
    finally:
        ctx.close()


def test_tune_rejects_bad_arguments(api_mod):
    import torch
    api = api_mod
    space = synth.tiny(1)
    say("tune bad arguments")
    ctx = api.Context(0)
    try:
        plan = api.plan_create(ctx, space.radix, torch.from_numpy(space.fitness_raw).cuda(), "hamming")
        with pytest.raises(api.FLError):
            api.tune(plan, sweeps=0)
        with pytest.raises(api.FLError):
            api.tune(plan, damping=1.5)
        plan.close()
    finally:
        ctx.close()


def test_bucket_mapping_is_tuned_and_used(api_mod):
    """The tuner's per-bucket mapping: rows per in-degree bucket exactly as the
    oracle's in-degrees give them, lanes per row and blocks per tile from the
    allowed sets; the binned layout then runs that mapping and matches the
    oracle."""
    import torch
    api = api_mod
    space = synth.mid()
    ctx = api.Context(0)
    try:
        say("bucket mapping, mid hamming")
        plan = api.plan_create(ctx, space.radix, torch.from_numpy(space.fitness_raw).cuda(), "hamming")
        before = api.bucket_map(plan)
        res = api.tune(plan, sweeps=3)
        after = res["buckets"]
        g = oracle.build_graph(space.radix, space.fitness_raw)
        deg = np.diff(g.row_ptr.astype(np.int64))
        edges = [0, 1, 2, 4, 8, 16, 32, 64, 1 << 40]
        for b, name in enumerate(api.BUCKETS):
            lo, hi = (0, 0) if b == 0 else (edges[b], edges[b + 1] - 1)
            want = int(np.count_nonzero((deg >= lo) & (deg <= hi)))
            assert after[name]["rows"] == before[name]["rows"] == want, (name, after[name], want)
            assert after[name]["lanes"] in (1, 2, 4, 8, 16, 32, 64) and after[name]["blocks"] in (1, 4)
        assert sum(v["rows"] for v in after.values()) == g.N
        assert -2 in res["us_per_sweep"] and res["us_per_sweep"][-2] > 0
        pr, mins, info = api.execute(plan, 0.85, 0.05, row_mapping=-2)
        assert info["row_mapping"] == -2
        o = oracle.analyze(space.radix, space.fitness_raw, oracle.HAMMING, 0.85, 0.05, tol=1e-12)
        assert np.array_equal(mins.cpu().numpy(), o.graph.minima)
        assert float(np.abs(pr.cpu().numpy() - o.pagerank).sum()) <= 1e-5
        plan.close()
    finally:
        ctx.close()
