"""GPU: exact PageRank by Jacobi sweeps to a fixed point (fl_execute_exact),
against the oracle's forward substitution in descending fitness order.

Valid for damping in (0, 1]; at d = 1, C_p is the probability that a
uniformly started random first-improvement descent ends within (1 + p) f_opt.
"""
import numpy as np
import pytest

import oracle
from paper_2210_01465_amd import synth

pytestmark = pytest.mark.gpu

NB = {"hamming": oracle.HAMMING, "adjacent": oracle.ADJACENT}


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


def _spaces():
    out = [synth.tiny(s) for s in range(3)] + [synth.mid()]
    out += [s for s in (synth.fuzz_space(j, max_params=6, max_radix=7, tie_levels=(3 if j % 3 == 0 else None))
                        for j in range(10)) if s.n_valid > 0 and s.n_raw <= 100_000]
    return out


@pytest.mark.parametrize("damping", [0.5, 0.85, 1.0])
@pytest.mark.parametrize("nb", ["hamming", "adjacent"])
def test_exact_matches_oracle(ctx, nb, damping):
    import torch
    from paper_2210_01465_amd import api
    for s in _spaces():
        say(f"exact {s.name} radix={s.radix} nb={nb} d={damping}")
        fit = torch.from_numpy(s.fitness_raw).cuda()
        plan = api.plan_create(ctx, s.radix, fit, nb)
        try:
            pr, mins, info = api.execute(plan, damping, 0.05, exact=True)
            pr = pr.cpu().numpy()
            mins = mins.cpu().numpy()
        finally:
            plan.close()
        g = oracle.build_graph(s.radix, s.fitness_raw, NB[nb])
        r, depth = g.dag_rank(damping)
        assert info["status"] == 0
        assert np.array_equal(mins, g.minima)
        l1 = float(np.abs(pr - r).sum())
        assert l1 <= 1e-5, (s.name, nb, damping, l1)
        assert abs(info["score"] - g.score(r, 0.05)[0]) <= 1e-5
        # settles after at most (longest path + 1) sweeps, seen by one more
        # sweep; sooner where the weight of a distant ancestor (d^k times the
        # product of 1/out_deg along the path) falls below FP32 resolution
        assert info["iterations"] <= depth + 2, (info["iterations"], depth)
        assert info["residual_l1"] == 0.0


def test_exact_agrees_with_power_iteration_and_layouts(ctx):
    import torch
    from paper_2210_01465_amd import api
    s = synth.mid()
    say("exact vs power iteration, every layout")
    fit = torch.from_numpy(s.fitness_raw).cuda()
    plan = api.plan_create(ctx, s.radix, fit, "hamming")
    try:
        ref, _, _ = api.execute(plan, 0.85, 0.05)   # FP32 sweeps, stopped at 2e-7
        ref = ref.cpu().numpy()
        outs = {}
        for lay in (-1, 1, 8):
            pr, _, info = api.execute(plan, 0.85, 0.05, row_mapping=lay, exact=True)
            outs[lay] = (pr.cpu().numpy(), info["iterations"])
        sep = {}
        for lay in (-1, 1):
            pr, _, info = api.execute(plan, 0.85, 0.05, row_mapping=lay, exact=True, separate_step=True)
            sep[lay] = (pr.cpu().numpy(), info["iterations"])
    finally:
        plan.close()
    assert float(np.abs(outs[-1][0] - ref).sum()) <= 2e-5
    # the slot sweep and the one-lane CSR sweep add in the same order; with a
    # step kernel per sweep the final scaling sums in the same order too
    assert np.array_equal(sep[-1][0], sep[1][0]) and sep[-1][1] == sep[1][1]
    # the lagged step makes the same sweeps: only the scaling's rounding differs
    for lay in (-1, 1):
        assert outs[lay][1] == sep[lay][1]
        assert float(np.abs(outs[lay][0] - sep[lay][0]).sum()) <= 1e-12
    assert float(np.abs(outs[8][0] - outs[-1][0]).sum()) <= 1e-5


def test_exact_errors(ctx):
    import torch
    from paper_2210_01465_amd import api, _abi
    s = synth.tiny(1)
    say("exact error paths")
    plan = api.plan_create(ctx, s.radix, torch.from_numpy(s.fitness_raw).cuda(), "hamming")
    try:
        for d in (0.0, 1.5, float("nan")):
            with pytest.raises(api.FLError) as e:
                api.execute(plan, d, 0.05, exact=True)
            assert e.value.status == _abi.FL_EINVAL
        with pytest.raises(api.FLError):
            api.execute(plan, 1.0, 0.05)                      # d = 1 only for the exact method
        pr, _, info = api.execute(plan, 0.85, 0.05, max_iter=2, exact=True, allow_noconv=True)
        assert info["status"] == _abi.FL_ENOCONV and info["iterations"] == 2
    finally:
        plan.close()
