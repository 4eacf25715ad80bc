"""GPU: the landscape figures around C_p, against the FP64 oracle.

* the C_p curve over p = 0, 1, ..., 15 % (Sec. VII-B) in one call;
* the naive metric f_opt / f(m) over the local minima (Sec. VII-A), exactly;
* plateau minima (sinks with an equal-fitness neighbour), exactly;
* the paper's failure convention (Sec. V): failed configurations kept as
  nodes with fitness 1e10, which creates large tie plateaus.
"""
import numpy as np
import pytest

import oracle
from paper_2210_01465_amd import synth

pytestmark = pytest.mark.gpu

NB = {"hamming": oracle.HAMMING, "adjacent": oracle.ADJACENT}
P_GRID = [j / 100 for j in range(16)]


def say(msg):
    print(f"[case] {msg}", flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2210_01465_amd import api
    c = api.Context(0)
    yield c
    c.close()


def _run(ctx, radix, f, nb, damping=0.85):
    import torch
    from paper_2210_01465_amd import api
    fit = torch.from_numpy(np.ascontiguousarray(f, dtype=np.float32)).cuda()
    plan = api.plan_create(ctx, radix, fit, nb)
    pr, mins, info = api.execute(plan, damping, 0.05)
    return plan, pr, mins, info


def _paper_mode(f):
    """Failed configurations (NaN) kept as nodes with fitness 1e10."""
    g = np.array(f, dtype=np.float32, copy=True)
    g[np.isnan(g)] = np.float32(1e10)
    return g


def _spaces():
    out = [(s.name, s.radix, s.fitness_raw) for s in (synth.tiny(0), synth.tiny(4), synth.mid())]
    out += [(s.name, s.radix, s.fitness_raw) for s in
            (synth.fuzz_space(j, max_params=5, max_radix=7, tie_levels=(3 if j % 2 else None)) for j in range(8))
            if s.n_valid > 0]
    return out


@pytest.mark.parametrize("nb", ["hamming", "adjacent"])
def test_score_curve_matches_oracle(ctx, nb):
    from paper_2210_01465_amd import api
    for name, radix, f in _spaces():
        say(f"C_p curve {name} radix={radix} nb={nb}")
        plan, pr, mins, info = _run(ctx, radix, f, nb)
        try:
            curve = api.score_curve(plan, pr, P_GRID)
            again = api.score_curve(plan, pr, [0.05])
        finally:
            plan.close()
        a = oracle.analyze(radix, f, NB[nb], 0.85, 0.05)
        ref = [a.graph.score(a.pagerank, p)[0] for p in P_GRID]
        assert np.allclose(curve, ref, rtol=0, atol=1e-5), (name, curve, ref)
        assert all(x <= y for x, y in zip(curve, curve[1:]))          # non-decreasing in p
        assert again[0] == curve[5] == info["score"]                   # same sums as fl_execute's C_p


def test_score_curve_saturates_and_rejects_bad_p(ctx):
    from paper_2210_01465_amd import api
    s = synth.mid()
    say("C_p curve saturation")
    plan, pr, mins, info = _run(ctx, s.radix, s.fitness_raw, "hamming")
    try:
        a = oracle.analyze(s.radix, s.fitness_raw, oracle.HAMMING, 0.85, 0.05)
        g = a.graph
        top = float(np.max(g.fit[g.minima])) / g.f_opt - 1.0
        assert api.score_curve(plan, pr, [top * (1 + 1e-9) + 1e-12, 10.0]) == [1.0, 1.0]
        for bad in ([-0.01], [float("nan")], [float("inf")]):
            with pytest.raises(api.FLError):
                api.score_curve(plan, pr, bad)
        with pytest.raises(api.FLError):
            api.score_curve(plan, pr, [])
    finally:
        plan.close()


@pytest.mark.parametrize("nb", ["hamming", "adjacent"])
def test_naive_metric_and_plateaus_exact(ctx, nb):
    from paper_2210_01465_amd import api
    for name, radix, f in _spaces():
        say(f"naive metric {name} radix={radix} nb={nb}")
        plan, pr, mins, info = _run(ctx, radix, f, nb)
        try:
            ratio, hist = api.naive_metric(plan, 20)
            ratio = ratio.cpu().numpy()
        finally:
            plan.close()
        g = oracle.build_graph(radix, f, NB[nb])
        ref, ref_hist = g.naive(20)           # the oracle's naive metric (Sec. VII-A), FP64
        assert np.array_equal(ratio, ref), name
        assert hist == ref_hist.tolist(), (name, hist, ref_hist)
        assert sum(hist) == g.M
        assert info["n_plateau"] == g.plateau_minima, (name, info["n_plateau"], g.plateau_minima)


@pytest.mark.parametrize("shape", range(4))
def test_paper_failure_mode(ctx, shape):
    """Sec. V keeps configurations that fail as points with fitness 1e10:
    they tie with each other (no edges among them), and a failed point with
    no valid neighbour is a plateau sink.  The four paper-shaped spaces with
    their failure rates, failures turned into 1e10, under both
    neighbourhoods."""
    from paper_2210_01465_amd import api
    s = synth.batched()[shape * 9]          # the first landscape of each paper shape
    f = _paper_mode(s.fitness_raw)
    for nb in ("hamming", "adjacent"):
        say(f"paper failure mode {s.name} radix={s.radix} nb={nb}")
        plan, pr, mins, info = _run(ctx, s.radix, f, nb)
        try:
            exp = {k: v.cpu().numpy() for k, v in api.plan_export(plan).items()}
            curve = api.score_curve(plan, pr, P_GRID)
            pr = pr.cpu().numpy()
            mins = mins.cpu().numpy()
        finally:
            plan.close()
        a = oracle.analyze(s.radix, f, NB[nb], 0.85, 0.05)
        g = a.graph
        assert info["n_valid"] == g.N and info["n_edges"] == g.E and info["n_minima"] == g.M
        assert np.array_equal(exp["row_ptr"], g.row_ptr) and np.array_equal(exp["col_idx"], g.col_idx)
        assert np.array_equal(mins, g.minima)
        assert info["n_plateau"] == g.plateau_minima
        assert float(np.abs(pr - a.pagerank).sum()) <= 1e-5
        ref = [g.score(a.pagerank, p)[0] for p in P_GRID]
        assert np.allclose(curve, ref, rtol=0, atol=1e-5)
