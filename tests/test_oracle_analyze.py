"""The oracle's one-call entry point (flo_analyze) against its step-by-step
functions: the same arithmetic in the same order, so every output is equal
bit for bit; plus its size and error contract.  CPU only."""
import numpy as np
import pytest

import oracle
from paper_2210_01465_amd import synth


def _spaces():
    out = [synth.tiny(s) for s in range(3)]
    out += [s for s in (synth.fuzz_space(j, max_params=5, max_radix=6, tie_levels=(3 if j % 2 else None))
                        for j in range(6)) if s.n_valid > 0]
    return out


@pytest.mark.parametrize("nb", [oracle.HAMMING, oracle.ADJACENT])
def test_one_call_equals_steps(nb):
    for s in _spaces():
        one = oracle.analyze_one_call(s.radix, s.fitness_raw, nb, 0.85, 0.05, tol=1e-12)
        g = oracle.build_graph(s.radix, s.fitness_raw, nb)
        r, it, res = g.pagerank(0.85, 1e-12, 1_000_000)
        score, num, den = g.score(r, 0.05)
        assert one["status"] == oracle.OK, s.name
        assert (one["n_raw"], one["N"], one["E"], one["M"], one["K"]) == (g.n_raw, g.N, g.E, g.M, g.K)
        assert one["plateau_minima"] == g.plateau_minima
        assert np.array_equal(one["valid_raw"], g.valid_raw)
        assert np.array_equal(one["row_ptr"], g.row_ptr)
        assert np.array_equal(one["col_idx"], g.col_idx)
        assert np.array_equal(one["minima"], g.minima)
        assert np.array_equal(one["pagerank"], r)
        assert one["iterations"] == it and one["residual"] == res
        assert (one["score"], one["mass_near"], one["mass_minima"]) == (score, num, den)
        assert one["f_opt"] == g.f_opt


def test_edge_capacity_and_errors():
    s = synth.tiny(0)
    full = oracle.analyze_one_call(s.radix, s.fitness_raw)
    assert full["status"] == oracle.OK and full["E"] > 0
    short = oracle.analyze_one_call(s.radix, s.fitness_raw, cap_edges=full["E"] - 1)
    assert short["status"] == oracle.ESIZE and short["E"] == full["E"] and "pagerank" not in short
    exact = oracle.analyze_one_call(s.radix, s.fitness_raw, cap_edges=full["E"])
    assert exact["status"] == oracle.OK and np.array_equal(exact["pagerank"], full["pagerank"])
    capped = oracle.analyze_one_call(s.radix, s.fitness_raw, max_iter=2)
    assert capped["status"] == oracle.ENOCONV and capped["iterations"] == 2 and "pagerank" in capped
    nan = oracle.analyze_one_call(s.radix, np.full(s.fitness_raw.shape, np.nan, np.float32))
    assert nan["status"] == oracle.EINVAL
    bad_d = oracle.analyze_one_call(s.radix, s.fitness_raw, damping=1.0)
    assert bad_d["status"] == oracle.EINVAL
