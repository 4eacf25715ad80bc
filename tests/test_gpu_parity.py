"""GPU parity: the HIP engine through the C ABI against the FP64 oracle.

Integer outputs (node map, CSR, out-degrees, minima, sizes) must match bit for
bit; PageRank within 1e-5 in L1 and C_p within 1e-5 absolute.  Every case
prints its name before touching the GPU so a failing run names it.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2210_01465_amd import synth

pytestmark = pytest.mark.gpu

NB = {"hamming": oracle.HAMMING, "adjacent": oracle.ADJACENT}
L1_TOL = 1e-5
SCORE_TOL = 1e-5


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.fixture(scope="module")
def ctx(torch_mod):
    from paper_2210_01465_amd import api
    c = api.Context(0)
    yield c
    c.close()


def say(msg):
    print(f"[case] {msg}", flush=True)


def _space(name, radix, f):
    return synth.Space(name, tuple(radix), np.asarray(f, dtype=np.float32).reshape(-1))


def run_gpu(ctx, space, nb, damping=0.85, p=0.05, row_mapping=0, tol=0.0, max_iter=0,
            allow_noconv=False):
    import torch
    from paper_2210_01465_amd import api
    fit = torch.from_numpy(np.ascontiguousarray(space.fitness_raw)).cuda()
    plan = api.plan_create(ctx, space.radix, fit, nb)
    try:
        ex = {k: v.cpu().numpy() for k, v in api.plan_export(plan).items()}
        pr, mins, info = api.execute(plan, damping, p, tol=tol, max_iter=max_iter,
                                     row_mapping=row_mapping, allow_noconv=allow_noconv)
        torch.cuda.synchronize()
        return ex, pr.cpu().numpy(), mins.cpu().numpy(), info, plan.sizes
    finally:
        plan.close()


def check_parity(ctx, space, nb, damping=0.85, p=0.05, row_mapping=0, ref=None):
    say(f"{space.name} radix={space.radix} nb={nb} d={damping} p={p} L={row_mapping}")
    ex, pr, mins, info, sizes = run_gpu(ctx, space, nb, damping, p, row_mapping)
    o = ref or oracle.analyze(space.radix, space.fitness_raw, NB[nb], damping, p)
    g = o.graph
    assert sizes["n_raw"] == g.n_raw and sizes["n_valid"] == g.N
    assert sizes["n_edges"] == g.E and sizes["n_minima"] == g.M
    assert sizes["f_opt"] == g.f_opt
    assert np.array_equal(ex["valid_raw"], g.valid_raw)
    assert np.array_equal(ex["row_ptr"], g.row_ptr)
    assert np.array_equal(ex["col_idx"], g.col_idx)
    assert np.array_equal(ex["out_deg"], g.out_deg)
    assert np.array_equal(mins, g.minima)
    l1 = float(np.abs(pr - o.pagerank).sum())
    assert l1 <= L1_TOL, (space.name, nb, l1)
    assert abs(info["score"] - o.score) <= SCORE_TOL, (info["score"], o.score)
    assert abs(info["mass_minima"] - o.mass_minima) <= SCORE_TOL
    assert abs(pr.sum() - 1.0) < 1e-9
    assert info["residual_l1"] < 2e-7 and info["status"] == 0
    return l1, info


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("nb", ["hamming", "adjacent"])
def test_tiny_parity(ctx, seed, nb):
    check_parity(ctx, synth.tiny(seed), nb)


@pytest.mark.parametrize("nb", ["hamming", "adjacent"])
def test_mid_parity(ctx, nb):
    check_parity(ctx, synth.mid(), nb)


@pytest.mark.parametrize("seed", range(40))
def test_fuzz_parity(ctx, seed):
    s = synth.fuzz_space(seed, max_params=7, max_radix=9,
                         tie_levels=(4 if seed % 3 == 0 else None))
    if s.n_valid == 0 or s.n_raw > 400_000:
        pytest.skip("no valid configuration" if s.n_valid == 0 else "larger than the fuzz cap")
    for nb in ("hamming", "adjacent"):
        check_parity(ctx, s, nb, damping=(0.5, 0.85, 0.9)[seed % 3], p=(0.0, 0.05, 0.15)[seed % 3])


ROWS_SLOTS = -1


@pytest.mark.parametrize("lanes", [ROWS_SLOTS, 1, 2, 4, 8, 16, 32, 64, -2])
def test_every_row_mapping(ctx, lanes):
    """Every sweep layout: the slot sweep, the CSR sweep with 1..64 lanes and
    the CSR sweep with rows binned by in-degree (-2)."""
    for nb in ("hamming", "adjacent"):
        check_parity(ctx, synth.tiny(3), nb, row_mapping=lanes)
        check_parity(ctx, synth.fuzz_space(5, max_params=6, max_radix=8), nb, row_mapping=lanes)
    check_parity(ctx, synth.mid(), "hamming", row_mapping=lanes)


def test_slot_layouts_agree_bit_for_bit(ctx):
    """The slot sweep reads the same x values as the one-lane CSR sweep and
    adds them in the same order: identical ranks.  The spaces cover waves
    straddling holes of excluded configurations, slot offsets from 1 to far
    beyond a wave's span, the most negative offset far below raw index 0,
    record widths 2 to 5, and both neighbourhoods."""
    import torch
    from paper_2210_01465_amd import api
    rng = np.random.default_rng(17)
    spaces = [synth.tiny(7), synth.mid()]
    spaces += [s for s in (synth.fuzz_space(j, max_params=6, max_radix=9, p_exclude=0.4) for j in range(30, 40))
               if s.n_valid > 0 and s.n_raw <= 300_000]
    for radix in ((3, 5, 2, 120), (60, 64), (120, 2), (2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 3)):
        n_raw = int(np.prod(radix))
        f = np.where(rng.random(n_raw) < 0.3, np.nan, rng.lognormal(0.0, 0.5, n_raw))
        spaces.append(_space(f"slots{radix}", radix, f))
    for s in spaces:
        for nb in ("hamming", "adjacent"):
            say(f"layouts agree {s.name} radix={s.radix} nb={nb}")
            fit = torch.from_numpy(np.ascontiguousarray(s.fitness_raw)).cuda()
            plan = api.plan_create(ctx, s.radix, fit, nb)
            try:
                if plan.sizes["mask_words"] == 0:
                    continue
                outs = {}
                for lay in (ROWS_SLOTS, 1):
                    for sep in (True, False):
                        pr, _, info = api.execute(plan, 0.85, 0.05, row_mapping=lay, separate_step=sep)
                        outs[lay, sep] = (pr.cpu().numpy(), info["iterations"])
                # with a step kernel per sweep the order of every sum is the same
                assert outs[ROWS_SLOTS, True][1] == outs[1, True][1]
                assert np.array_equal(outs[ROWS_SLOTS, True][0], outs[1, True][0]), (s.name, nb)
                # the lagged step sums per workgroup, whose count depends on
                # the kernel: the same iterates up to rounding
                for lay in (ROWS_SLOTS, 1):
                    assert abs(outs[lay, False][1] - outs[lay, True][1]) <= 1
                    assert float(np.abs(outs[lay, False][0] - outs[lay, True][0]).sum()) <= L1_TOL
            finally:
                plan.close()


def test_mask_widths(ctx):
    """Candidate slots K' = 2 sum(r - 1): 128 (three record words), 130,
    256 (five words, the most a record holds) and 258 (generic kernels, CSR
    sweep only), for Hamming; adjacent stays small."""
    rng = np.random.default_rng(5)
    for radix in ((33, 33), (34, 33), (65, 65), (65, 66), (129,), (130,)):
        n_raw = int(np.prod(radix))
        f = np.where(rng.random(n_raw) < 0.1, np.nan, rng.random(n_raw) + 0.5)
        s = _space(f"K{sum(r - 1 for r in radix)}", radix, f)
        for nb in ("hamming", "adjacent"):
            check_parity(ctx, s, nb)




def test_slot_sweep_plain_loads(ctx):
    """A raw-index span of 2^29 or more (here 28 binary parameters, 2^28 raw
    configurations, neighbours up to 2^27 away) does not fit the buffer-load
    offsets, so the slot sweep takes its plain-load form.  The valid points
    form a 2^18-point sub-cube (bits 10..19 zero) with 10 % failures, so every
    parameter, the most significant included, has in-edges.  Checked against
    the one-lane CSR sweep on the same plan (same order of addition with a
    step kernel per sweep: equal bit for bit), the lagged step against that,
    and against the invariants of a probability vector with teleport (sum 1,
    r >= (1 - d)/N)."""
    import torch
    from paper_2210_01465_amd import api
    n_raw = 1 << 28
    rng = np.random.default_rng(29)
    idx = ((np.arange(256, dtype=np.int64) << 20)[:, None] | np.arange(1024, dtype=np.int64)[None, :]).ravel()
    idx = idx[rng.random(idx.size) >= 0.1]
    f = np.full(n_raw, np.nan, np.float32)
    f[idx] = rng.lognormal(0.0, 0.5, idx.size).astype(np.float32)
    say(f"plain-load slot sweep: 2^28 raw, {idx.size} valid")
    plan = api.plan_create(ctx, (2,) * 28, torch.from_numpy(f).cuda(), "hamming")
    del f
    try:
        assert plan.sizes["mask_words"] == 2 and plan.n_valid == idx.size
        pr_s, mins_s, info_s = api.execute(plan, 0.85, 0.05, row_mapping=ROWS_SLOTS, separate_step=True)
        pr_c, mins_c, info_c = api.execute(plan, 0.85, 0.05, row_mapping=1, separate_step=True)
        pr_s, pr_c = pr_s.cpu().numpy(), pr_c.cpu().numpy()
        assert info_s["iterations"] == info_c["iterations"] and info_s["status"] == 0
        assert np.array_equal(pr_s, pr_c)
        pr_l, mins_l, info_l = api.execute(plan, 0.85, 0.05, row_mapping=ROWS_SLOTS)
        assert abs(info_l["iterations"] - info_s["iterations"]) <= 1 and info_l["status"] == 0
        assert float(np.abs(pr_l.cpu().numpy() - pr_s).sum()) <= L1_TOL
        assert np.array_equal(mins_l.cpu().numpy(), mins_s.cpu().numpy())
        assert np.array_equal(mins_s.cpu().numpy(), mins_c.cpu().numpy())
        assert info_s["n_edges"] > 0 and abs(pr_s.sum() - 1.0) <= 1e-6
        assert pr_s.min() >= (1.0 - 0.85) / idx.size * (1.0 - 1e-5)
    finally:
        plan.close()


def test_edge_cases(ctx):
    rng = np.random.default_rng(0)
    cases = [
        _space("single_valid", (3,), [np.nan, 2.0, np.inf]),
        _space("two_nodes", (2,), [1.0, 2.0]),
        _space("all_equal", (4, 3, 5), np.ones(60)),
        _space("radix_one_dims", (1, 7, 1, 3, 1), rng.random(21) + 0.5),
        _space("complete_graph_1d", (1000,), rng.permutation(1000) + 1.0),
        _space("ragged_tail", (257,), rng.random(257) + 0.5),
        _space("tiles_and_tail", (3, 5, 7, 11, 13), rng.random(15015) + 0.5),
        _space("many_ties", (6, 6, 6), rng.integers(1, 3, 216).astype(np.float64)),
        _space("mostly_excluded", (50, 40), np.where(rng.random(2000) < 0.9, np.nan,
                                                      rng.random(2000) + 0.5)),
    ]
    for s in cases:
        for nb in ("hamming", "adjacent"):
            check_parity(ctx, s, nb)


@pytest.mark.parametrize("nb", ["hamming", "adjacent"])
def test_paper_shapes(ctx, nb):
    """The paper's four kernel-space shapes with its average failed counts."""
    spaces = synth.batched()
    for s in spaces[0:36:9]:
        check_parity(ctx, s, nb)


def test_determinism(ctx):
    s = synth.mid()
    a = run_gpu(ctx, s, "hamming")
    b = run_gpu(ctx, s, "hamming")
    for k in a[0]:
        assert np.array_equal(a[0][k], b[0][k])
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert a[3]["score"] == b[3]["score"] and a[3]["iterations"] == b[3]["iterations"]


def test_plan_reuse_other_damping(ctx):
    """One FFG, several (d, p): only the PageRank and the score change."""
    import torch
    from paper_2210_01465_amd import api
    s = synth.tiny(4)
    fit = torch.from_numpy(s.fitness_raw).cuda()
    plan = api.plan_create(ctx, s.radix, fit, "hamming")
    try:
        g = oracle.build_graph(s.radix, s.fitness_raw)
        for d, p in ((0.8, 0.0), (0.85, 0.05), (0.9, 0.15), (0.5, 1.0)):
            say(f"plan reuse d={d} p={p}")
            pr, mins, info = api.execute(plan, d, p)
            r, _, _ = g.pagerank(d)
            sc, _, _ = g.score(r, p)
            assert float(np.abs(pr.cpu().numpy() - r).sum()) <= L1_TOL
            assert abs(info["score"] - sc) <= SCORE_TOL
    finally:
        plan.close()


def test_error_paths(ctx):
    import torch
    from paper_2210_01465_amd import api, _abi
    say("error paths")
    ones = torch.ones(8, device="cuda")
    for bad in (0.0, -1.0, -math.inf):
        f = ones.clone()
        f[3] = bad
        with pytest.raises(api.FLError) as e:
            api.plan_create(ctx, (8,), f)
        assert e.value.status == _abi.FL_EINVAL
    with pytest.raises(api.FLError) as e:
        api.plan_create(ctx, (8,), torch.full((8,), float("nan"), device="cuda"))
    assert e.value.status == _abi.FL_EINVAL
    with pytest.raises(api.FLError) as e:
        api.plan_create(ctx, (2, 0, 4), torch.ones(0, device="cuda"))
    assert e.value.status == _abi.FL_EINVAL
    import ctypes
    lib = _abi.load()
    one = torch.ones(1, device="cuda")
    for n_params in (0, 33):
        radix = (ctypes.c_int32 * 33)(*([1] * 33))
        sp = _abi.fl_space(n_params, ctypes.cast(radix, ctypes.POINTER(ctypes.c_int32)))
        h = ctypes.c_void_p()
        rc = lib.fl_plan_create(ctx.handle, ctypes.byref(sp), ctypes.c_void_p(one.data_ptr()), 0,
                                ctypes.byref(h), None)
        assert rc == _abi.FL_EINVAL, n_params
    with pytest.raises(ValueError):
        api.plan_create(ctx, (3, 3), torch.ones(8, device="cuda"))  # wrong size, host check
    plan = api.plan_create(ctx, (8,), ones)
    try:
        for kw in ({"damping": 0.0}, {"damping": 1.0}, {"damping": float("nan")},
                   {"p": -0.1}, {"p": float("inf")}, {"row_mapping": 3}, {"row_mapping": -3},
                   {"max_iter": -1}):
            args = {"damping": 0.85, "p": 0.05}
            args.update(kw)
            with pytest.raises(api.FLError) as e:
                api.execute(plan, **args)
            assert e.value.status == _abi.FL_EINVAL, kw
        # unknown flags and a non-zero reserved field
        out = torch.empty(8, dtype=torch.float64, device="cuda")
        mins = torch.empty(8, dtype=torch.int32, device="cuda")
        for flags, reserved in ((2, 0), (-1, 0), (0, 1)):
            prm = _abi.fl_params(0.85, 0.05, 0.0, 0, 0, flags, reserved)
            rc = lib.fl_execute(ctx.handle, plan.handle, ctypes.byref(prm), ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(mins.data_ptr()), None)
            assert rc == _abi.FL_EINVAL, (flags, reserved)
    finally:
        plan.close()
    wide = api.plan_create(ctx, (200,), torch.arange(1, 201, dtype=torch.float32, device="cuda"))
    try:
        with pytest.raises(api.FLError) as e:
            api.execute(wide, row_mapping=ROWS_SLOTS)
        assert e.value.status == _abi.FL_EINVAL
    finally:
        wide.close()


def test_overflow_rejected_before_any_launch(ctx):
    import ctypes
    from paper_2210_01465_amd import _abi
    say("overflow")
    lib = _abi.load()
    radix = (ctypes.c_int32 * 2)(1 << 16, 1 << 15)
    sp = _abi.fl_space(2, ctypes.cast(radix, ctypes.POINTER(ctypes.c_int32)))
    h = ctypes.c_void_p()
    # a non-null dummy pointer: the call must fail on the size before reading it
    rc = lib.fl_plan_create(ctx.handle, ctypes.byref(sp), ctypes.c_void_p(16), 0,
                            ctypes.byref(h), None)
    assert rc == _abi.FL_EOVERFLOW


def test_iteration_cap_reports_noconv(ctx):
    from paper_2210_01465_amd import _abi
    s = synth.mid()
    say("max_iter=3")
    ex, pr, mins, info, sizes = run_gpu(ctx, s, "hamming", max_iter=3, allow_noconv=True)
    assert info["status"] == _abi.FL_ENOCONV and info["iterations"] == 3
    assert info["residual_l1"] > 2e-7
    # outputs are written: the 3-step FP64 oracle iterate agrees
    g = oracle.build_graph(s.radix, s.fitness_raw)
    r, it, _ = g.pagerank(0.85, 0.0, 3, check=False)
    assert it == 3 and float(np.abs(pr - r).sum()) <= L1_TOL
    assert np.array_equal(mins, g.minima)


def test_analyze_one_shot(ctx):
    import torch
    from paper_2210_01465_amd import api
    s = synth.tiny(7)
    say("fl_analyze")
    res = api.analyze(s.radix, torch.from_numpy(s.fitness_raw).cuda(), "adjacent", 0.9, 0.1,
                      ctx=ctx)
    o = oracle.analyze(s.radix, s.fitness_raw, oracle.ADJACENT, 0.9, 0.1)
    assert np.array_equal(res.valid_raw.cpu().numpy(), o.graph.valid_raw)
    assert np.array_equal(res.minima.cpu().numpy(), o.graph.minima)
    assert float(np.abs(res.pagerank.cpu().numpy() - o.pagerank).sum()) <= L1_TOL
    assert abs(res.score - o.score) <= SCORE_TOL


@pytest.fixture(scope="module")
def large_ref():
    s = synth.large()
    return s, oracle.analyze(s.radix, s.fitness_raw, oracle.HAMMING, 0.85, 0.05)


def test_large_parity_full_size(ctx, large_ref):
    """1.5 M valid configurations, Hamming, in the launch configuration the
    benchmark times (automatic row mapping)."""
    s, ref = large_ref
    l1, info = check_parity(ctx, s, "hamming", ref=ref)
    print(f"large: L1={l1:.3e} iterations={info['iterations']} lanes={info['row_mapping']}")
