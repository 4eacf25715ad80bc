"""Checks that pin the oracle to facts other than itself.

Each ``check_*`` raises AssertionError on a mismatch.  They take the path of
an oracle library so that the same checks can be run against copies of the
oracle with a planted mistake (see test_oracle_mutants.py).
"""
from __future__ import annotations

import itertools
import math
import os

import numpy as np

import oracle
from brute import BruteFFG, configs, dag_pagerank, grid_degrees, kahn_acyclic
from paper_2210_01465_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
NB = {"hamming": oracle.HAMMING, "adjacent": oracle.ADJACENT}
# enough for tol 1e-14 at d = 0.99 on the small cases; a broken iteration that
# does not converge fails fast instead of running to a million steps
MAX_ITER = 20000


def _golden_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([c.strip() for c in line.split("|")])
    return rows


def small_cases():
    """Config-1 landscapes, plus random small spaces with and without ties."""
    cases = []
    for seed in range(4):
        s = synth.tiny(seed)
        cases.append((s.radix, s.fitness_raw))
    seed = 0
    while len(cases) < 28:
        s = synth.fuzz_space(seed, max_params=5, max_radix=5,
                             tie_levels=(3 if seed % 2 else None))
        seed += 1
        if s.n_raw <= 300:
            cases.append((s.radix, s.fitness_raw))
    return cases


def check_paper_sizes(lib):
    """Table 2 #points = product of the appendix value-list lengths."""
    for name, radices, points in _golden_rows("paper_space_sizes.txt"):
        radix = [int(r) for r in radices.split()]
        g = oracle.build_graph(radix, np.ones(int(points), np.float32), lib_path=lib)
        assert g.n_raw == int(points), (name, g.n_raw, points)
        assert g.N == int(points) and g.E == 0 and g.M == g.N, name
        assert g.K == sum(r - 1 for r in radix), name


def check_adjacent_example(lib):
    """Sec. III-B worked example of the adjacent neighbourhood."""
    for values, value, expect in _golden_rows("adjacent_example.txt"):
        vals = [int(v) for v in values.split()]
        want = sorted(int(v) for v in expect.split())
        g = oracle.build_graph([len(vals)], np.ones(len(vals), np.float32),
                               oracle.ADJACENT, lib_path=lib)
        got = sorted(vals[j] for j in g.neighbours(vals.index(int(value))))
        assert got == want, (value, got, want)
        h = oracle.build_graph([len(vals)], np.ones(len(vals), np.float32),
                               oracle.HAMMING, lib_path=lib)
        got_h = sorted(vals[j] for j in h.neighbours(vals.index(int(value))))
        assert got_h == sorted(v for v in vals if v != int(value))


def check_neighbours_product_order(lib):
    """Neighbour raw indices agree with digit tuples in itertools.product order."""
    for radix in [(3, 1, 4), (2, 3, 2, 2), (5,), (1, 1), (4, 2, 3)]:
        n_raw = int(np.prod(radix))
        cfg = configs(radix)
        for nb in ("hamming", "adjacent"):
            g = oracle.build_graph(radix, np.ones(n_raw, np.float32), NB[nb], lib_path=lib)
            for i in range(n_raw):
                want = []
                for j in range(n_raw):
                    diff = [k for k in range(len(radix)) if cfg[i][k] != cfg[j][k]]
                    if len(diff) == 1 and (nb == "hamming" or abs(cfg[i][diff[0]] - cfg[j][diff[0]]) == 1):
                        want.append(j)
                assert list(g.neighbours(i)) == want, (radix, nb, i)


def check_ffg_bruteforce(lib, cases=None):
    """CSR, degrees, minima and f_opt against all-pairs brute force."""
    for radix, fit in (cases or small_cases()):
        if not np.any(np.isfinite(fit) & (fit > 0)):
            continue
        for nb in ("hamming", "adjacent"):
            b = BruteFFG(radix, fit, nb)
            g = oracle.build_graph(radix, fit, NB[nb], lib_path=lib)
            rp, col = b.csr()
            assert g.N == b.N and g.E == b.E and g.M == len(b.minima), (radix, nb)
            assert np.array_equal(g.valid_raw, b.raw)
            assert np.array_equal(g.row_ptr, rp), (radix, nb)
            assert np.array_equal(g.col_idx, col), (radix, nb)
            assert np.array_equal(g.out_deg, b.out_deg), (radix, nb)
            assert np.array_equal(g.minima, b.minima), (radix, nb)
            assert g.f_opt == b.f_opt
            assert kahn_acyclic(g.N, g.row_ptr, g.col_idx)


def check_pagerank_dense(lib, cases=None, dampings=(0.5, 0.85, 0.9, 0.99)):
    """Oracle PageRank against a dense linear solve and a dense eigenvector."""
    for radix, fit in (cases or small_cases()):
        if not np.any(np.isfinite(fit) & (fit > 0)):
            continue
        b = BruteFFG(radix, fit, "hamming")
        g = oracle.build_graph(radix, fit, oracle.HAMMING, lib_path=lib)
        for d in dampings:
            r, _, _ = g.pagerank(d, 1e-14, MAX_ITER)
            rs = b.pagerank_solve(d)
            assert np.abs(r - rs).sum() <= 1e-11, (radix, d, np.abs(r - rs).sum())
            if b.N <= 400:
                re = b.pagerank_eig(d)
                assert np.abs(r - re).sum() <= 1e-10, (radix, d)


def check_closed_forms(lib):
    """PageRank closed forms on 1-D spaces (derivations in the docstrings of brute.dag_pagerank)."""
    for d in (0.5, 0.85, 0.9):
        # two nodes, f0 < f1: r = ((1+d)/(2+d), 1/(2+d))
        g = oracle.build_graph([2], np.array([1.0, 2.0], np.float32), lib_path=lib)
        r, _, _ = g.pagerank(d, 1e-13, MAX_ITER)
        assert abs(r[0] - (1 + d) / (2 + d)) < 1e-13 and abs(r[1] - 1 / (2 + d)) < 1e-13
        # adjacent chain, f increasing with the index: u_i = (1 - d^(m-i))/(1-d)
        m = 9
        g = oracle.build_graph([m], np.arange(1, m + 1, dtype=np.float32),
                               oracle.ADJACENT, lib_path=lib)
        r, _, _ = g.pagerank(d, 1e-13, MAX_ITER)
        u = np.array([(1 - d ** (m - i)) / (1 - d) for i in range(m)])
        assert np.abs(r - u / u.sum()).sum() < 1e-12
        assert g.E == m - 1 and list(g.minima) == [0]
        # Hamming on one parameter = complete graph; rank j (0 = best):
        # u_j = prod_{l=j+1}^{m-1} (1 + d/l)
        perm = np.random.default_rng(3).permutation(m)
        f = (perm + 1).astype(np.float32)          # node i has rank perm[i]
        g = oracle.build_graph([m], f, oracle.HAMMING, lib_path=lib)
        r, _, _ = g.pagerank(d, 1e-13, MAX_ITER)
        uj = np.array([math.prod(1 + d / l for l in range(j + 1, m)) for j in range(m)])
        u = uj[perm]
        assert np.abs(r - u / u.sum()).sum() < 1e-12
        assert g.E == m * (m - 1) // 2 and g.M == 1


def check_separable_minima(lib):
    """f = prod_i g_i(x_i), g_i a permutation of 1..r_i (exact in float32):
    Hamming has exactly one minimum; adjacent has prod_i (#1-D minima of g_i)."""
    rng = np.random.default_rng(11)
    for _ in range(12):
        n = int(rng.integers(1, 6))
        radix = tuple(int(r) for r in rng.integers(2, 8, size=n))
        gs = [rng.permutation(r) + 1 for r in radix]
        f = np.ones(radix, dtype=np.float64)
        for i, gi in enumerate(gs):
            shape = [1] * n
            shape[i] = radix[i]
            f = f * gi.reshape(shape)
        f = f.astype(np.float32).reshape(-1)
        h = oracle.build_graph(radix, f, oracle.HAMMING, lib_path=lib)
        assert h.M == 1 and f[h.valid_raw[h.minima[0]]] == f.min()
        a = oracle.build_graph(radix, f, oracle.ADJACENT, lib_path=lib)

        def local_min_1d(gi):
            return sum(1 for k in range(len(gi))
                       if (k == 0 or gi[k - 1] > gi[k]) and (k == len(gi) - 1 or gi[k + 1] > gi[k]))
        assert a.M == math.prod(local_min_1d(gi) for gi in gs), (radix, a.M)
        s, _, _ = h.score(h.pagerank(0.85, 1e-13, MAX_ITER)[0], 0.0)
        assert s == 1.0


def _tie_cases():
    """Small spaces with many exact ties: the fuzz spaces drawn from a few
    fitness levels, and config-1 landscapes in the paper's failure mode
    (failed and constraint-violating configurations kept as points of
    fitness 1e10, Sec. V), where every failed point ties with the others."""
    cases = [(r, f) for r, f in small_cases() if np.unique(f[np.isfinite(f)]).size < f.size]
    for seed in range(3):
        s = synth.tiny(seed)
        f = np.array(s.fitness_raw, dtype=np.float32, copy=True)
        f[~np.isfinite(f)] = np.float32(1e10)
        cases.append((s.radix, f))
    return cases


def check_plateau_minima(lib):
    """Plateau minima (sinks with a valid neighbour of exactly equal fitness)
    counted from the brute-force neighbour lists of digit tuples: every
    minimum of BruteFFG is looked at, its valid neighbours compared for
    equality; excluded points (NaN / +inf) are not neighbours."""
    seen_plateau = 0
    for radix, fit in _tie_cases():
        if not np.any(np.isfinite(fit) & (fit > 0)):
            continue
        for nb in ("hamming", "adjacent"):
            b = BruteFFG(radix, fit, nb)
            want = sum(1 for v in b.minima if any(b.f[w] == b.f[v] for w in b.nbrs[v]))
            g = oracle.build_graph(radix, fit, NB[nb], lib_path=lib)
            assert g.plateau_minima == want, (radix, nb, g.plateau_minima, want)
            seen_plateau += want
    assert seen_plateau > 0          # the cases do exercise plateaus


def check_naive_separable(lib):
    """Naive metric (Sec. VII-A) on separable power-of-two landscapes:
    f = 2^(e_0(x_0) + ... + e_{n-1}(x_{n-1})) with distinct exponents per
    parameter is exact in float32, neighbours never tie, and under the
    adjacent neighbourhood the minima are exactly the digit tuples whose
    every digit is a 1-D local minimum of its e_i.  So the ratios
    f_opt / f(m) form the multiset {2^(sum_i min e_i - e_i(a_i))} over those
    tuples, each an exact binary fraction, and their histogram is fixed."""
    rng = np.random.default_rng(23)
    for _ in range(10):
        n = int(rng.integers(1, 5))
        radix = tuple(int(r) for r in rng.integers(2, 7, size=n))
        es = [rng.permutation(r) for r in radix]          # distinct exponents 0..r-1
        grid = np.zeros(radix, dtype=np.int64)
        for i, ei in enumerate(es):
            shape = [1] * n
            shape[i] = radix[i]
            grid = grid + ei.reshape(shape)
        f = np.ldexp(np.float32(1.0), grid.reshape(-1)).astype(np.float32)
        local = [[k for k in range(len(ei))
                  if (k == 0 or ei[k - 1] > ei[k]) and (k == len(ei) - 1 or ei[k + 1] > ei[k])]
                 for ei in es]
        want = sorted(2.0 ** -sum(int(es[i][a[i]]) - int(es[i].min()) for i in range(n))
                      for a in itertools.product(*local))
        for n_bins in (1, 4, 20):
            g = oracle.build_graph(radix, f, oracle.ADJACENT, lib_path=lib)
            ratio, hist = g.naive(n_bins)
            assert sorted(ratio.tolist()) == want, (radix, ratio, want)
            want_hist = [0] * n_bins
            for q in want:                    # exact binary fractions: floor is exact
                want_hist[min(int(q * n_bins), n_bins - 1)] += 1
            assert hist.tolist() == want_hist, (radix, n_bins, hist, want_hist)
            # the ratios follow the minima in ascending node id
            assert np.array_equal(ratio, g.f_opt / g.fit[g.minima].astype(np.float64))
        # Hamming: the single minimum is the optimum, ratio exactly 1, last bin
        h = oracle.build_graph(radix, f, oracle.HAMMING, lib_path=lib)
        ratio, hist = h.naive(20)
        assert ratio.tolist() == [1.0] and hist[-1] == 1 and hist.sum() == 1


def check_score_brute(lib, cases=None):
    """C_p recomputed from the brute minima with the <= (1+p) f_opt rule;
    non-decreasing in p; 1 once p reaches max_L f / f_opt - 1."""
    for radix, fit in (cases or small_cases()):
        if not np.any(np.isfinite(fit) & (fit > 0)):
            continue
        b = BruteFFG(radix, fit, "hamming")
        g = oracle.build_graph(radix, fit, oracle.HAMMING, lib_path=lib)
        r, _, _ = g.pagerank(0.85, 1e-13, MAX_ITER)
        prev = -1.0
        for p in [0.0, 0.01, 0.02, 0.05, 0.1, 0.15, 0.5]:
            s, num, den = g.score(r, p)
            t = (1.0 + p) * b.f_opt
            want_num = sum(r[m] for m in b.minima if float(b.f[m]) <= t)
            want_den = sum(r[m] for m in b.minima)
            assert abs(num - want_num) <= 1e-15 and abs(den - want_den) <= 1e-15
            assert s >= prev
            prev = s
        # C_p = 1 once p >= max_L f / f_opt - 1 (nudged past the FP64 rounding
        # of (1+p)*f_opt at the exact boundary)
        p_sat = max(float(b.f[m]) for m in b.minima) / b.f_opt - 1.0
        assert g.score(r, p_sat + 1e-12)[0] == 1.0
        # p = 0: exactly the minima tied with the optimum
        tied = [m for m in b.minima if float(b.f[m]) == b.f_opt]
        s0 = g.score(r, 0.0)[0]
        assert abs(s0 - sum(r[m] for m in tied) / sum(r[m] for m in b.minima)) <= 1e-15


def check_dag_identity(lib, spaces, nbs=("hamming",), d=0.85):
    """Oracle power iteration against the exact DAG solve r = u/sum(u), (I-dP)u = 1."""
    for s in spaces:
        for nb in nbs:
            g = oracle.build_graph(s.radix, s.fitness_raw, NB[nb], lib_path=lib)
            r, _, _ = g.pagerank(d, 1e-13, MAX_ITER)
            ref = dag_pagerank(g.N, g.row_ptr, g.col_idx, g.out_deg, d)
            assert np.abs(r - ref).sum() <= 1e-12, (s.name, nb, np.abs(r - ref).sum())


def _absorption(g, target):
    """Probability that a descent from node v, moving to a uniformly random
    strictly better neighbour until none exists, stops in a node of
    ``target``; by dynamic programming over ascending fitness (the
    definition written out, no matrix algebra)."""
    out = [[] for _ in range(g.N)]
    for w in range(g.N):
        for e in range(g.row_ptr[w], g.row_ptr[w + 1]):
            out[int(g.col_idx[e])].append(w)      # edge col_idx[e] -> w
    q = np.zeros(g.N)
    tgt = np.zeros(g.N, dtype=bool)
    tgt[list(target)] = True
    for v in np.argsort(g.fit, kind="stable"):   # better nodes first
        q[v] = float(tgt[v]) if not out[v] else sum(q[w] for w in out[v]) / len(out[v])
    return q


def _longest_path(g):
    level = np.zeros(g.N, dtype=np.int64)
    for w in np.argsort(-g.fit, kind="stable"):   # worse nodes first
        a, b = g.row_ptr[w], g.row_ptr[w + 1]
        if b > a:
            level[w] = 1 + level[g.col_idx[a:b]].max()
    return int(level.max()) if g.N else 0


def check_dag_rank(lib, cases=None):
    """The oracle's exact rank (forward substitution in descending fitness)
    against the Jacobi sweep u <- 1 + d P u of brute.dag_pagerank at
    d = 0.5, 0.85 and 1, against the oracle's power iteration at d < 1, its
    reported depth against the longest path, and at d = 1 its C_p against the
    probability that a uniformly started random descent ends in L_p."""
    for radix, f in (cases or small_cases()):
        if not np.any(np.isfinite(f) & (f > 0)):
            continue
        for nb in ("hamming", "adjacent"):
            g = oracle.build_graph(radix, f, NB[nb], lib_path=lib)
            for d in (0.5, 0.85, 1.0):
                r, depth = g.dag_rank(d)
                ref = dag_pagerank(g.N, g.row_ptr, g.col_idx, g.out_deg, d)
                assert np.abs(r - ref).sum() <= 1e-12, (radix, nb, d)
                if d < 1.0:
                    rp, _, _ = g.pagerank(d, 1e-13, MAX_ITER)
                    assert np.abs(r - rp).sum() <= 1e-11, (radix, nb, d)
            assert depth == _longest_path(g), (radix, nb)
            for p in (0.0, 0.05, 0.3):
                near = [int(m) for m in g.minima if float(g.fit[m]) <= (1.0 + p) * g.f_opt]
                prob = _absorption(g, near).mean()
                assert abs(g.score(r, p)[0] - prob) <= 1e-12, (radix, nb, p)


def check_grid_degrees(lib, spaces, nbs=("hamming", "adjacent")):
    """Per-node in/out degree, E and minima against whole-array comparisons."""
    for s in spaces:
        for nb in nbs:
            g = oracle.build_graph(s.radix, s.fitness_raw, NB[nb], lib_path=lib)
            ind, outd, valid = grid_degrees(s.radix, s.fitness_raw, nb)
            ind, outd, valid = ind.reshape(-1), outd.reshape(-1), valid.reshape(-1)
            assert np.array_equal(np.flatnonzero(valid), g.valid_raw)
            assert np.array_equal(np.diff(g.row_ptr.astype(np.int64)), ind[g.valid_raw])
            assert np.array_equal(g.out_deg, outd[g.valid_raw])
            assert g.E == int(outd.sum()) == int(ind.sum())
            assert np.array_equal(g.minima, np.flatnonzero(outd[g.valid_raw] == 0))
            # every edge strictly decreases fitness, hence the FFG is acyclic
            rows = np.repeat(np.arange(g.N), np.diff(g.row_ptr))
            assert np.all(g.fit[g.col_idx] > g.fit[rows])
            assert g.f_opt == float(s.fitness_raw[valid.nonzero()[0]].min())


def check_invariants(lib, spaces, d=0.85):
    """r >= (1-d)/N, sum r = 1, ||G r - r||_1 small, ranks sum to 1."""
    import scipy.sparse as sp
    for s in spaces:
        g = oracle.build_graph(s.radix, s.fitness_raw, lib_path=lib)
        r, _, _ = g.pagerank(d, 1e-13, MAX_ITER)
        N = g.N
        assert abs(r.sum() - 1.0) < 1e-12
        assert np.all(r >= (1 - d) / N * (1 - 1e-12))
        rows = np.repeat(np.arange(N), np.diff(g.row_ptr))
        deg = g.out_deg.astype(np.float64)
        P = sp.csr_matrix((1.0 / deg[g.col_idx], (rows, g.col_idx)), shape=(N, N))
        sink = g.out_deg == 0
        Gr = d * (P @ r) + (d * r[sink].sum() + (1 - d) * r.sum()) / N
        assert np.abs(Gr - r).sum() < 1e-12


def check_metamorphic(lib):
    """f -> 2f changes nothing but f_opt; permuting the parameters permutes the outputs."""
    for seed in range(3):
        s = synth.tiny(seed)
        a = oracle.analyze(s.radix, s.fitness_raw, max_iter=MAX_ITER, lib_path=lib)
        b = oracle.analyze(s.radix, s.fitness_raw * np.float32(2), max_iter=MAX_ITER, lib_path=lib)
        ga, gb = a.graph, b.graph
        for name in ("valid_raw", "row_ptr", "col_idx", "out_deg", "minima"):
            assert np.array_equal(getattr(ga, name), getattr(gb, name)), name
        assert np.array_equal(a.pagerank, b.pagerank) and a.score == b.score
        assert gb.f_opt == 2 * ga.f_opt
        for perm in itertools.permutations(range(len(s.radix))):
            grid = s.fitness_raw.reshape(s.radix)
            pgrid = np.ascontiguousarray(np.transpose(grid, perm))
            c = oracle.analyze(pgrid.shape, pgrid.reshape(-1), max_iter=MAX_ITER, lib_path=lib)
            # map each node of the permuted space back to its original raw index
            dig = np.array(np.unravel_index(c.graph.valid_raw, pgrid.shape))
            orig = np.zeros_like(dig)
            orig[list(perm)] = dig
            raw = np.ravel_multi_index(tuple(orig), s.radix)
            pos = np.searchsorted(ga.valid_raw, raw)
            assert np.array_equal(ga.valid_raw[pos], raw)
            assert np.abs(a.pagerank[pos] - c.pagerank).sum() < 1e-12
            assert sorted(pos[c.graph.minima]) == list(ga.minima)
            assert abs(a.score - c.score) < 1e-12 and ga.E == c.graph.E


def check_errors(lib):
    """Invalid inputs are rejected; N = 1 is a single sink with rank 1."""
    one = np.ones(4, np.float32)
    for bad in (0.0, -1.0, -np.inf):
        f = one.copy()
        f[2] = bad
        try:
            oracle.build_graph([4], f, lib_path=lib)
        except oracle.OracleError as e:
            assert e.code == oracle.EINVAL
        else:
            raise AssertionError(f"fitness {bad} accepted")
    for radix, f in (([4], np.full(4, np.nan, np.float32)), ([0], one[:0]), ([], one[:1]),
                     ([1] * 33, one[:1])):
        try:
            oracle.build_graph(radix, f, lib_path=lib)
        except oracle.OracleError as e:
            assert e.code == oracle.EINVAL
        else:
            raise AssertionError(f"{radix} accepted")
    try:
        oracle.build_graph([1 << 16, 1 << 15], one, lib_path=lib)
    except oracle.OracleError as e:
        assert e.code == oracle.EOVERFLOW
    else:
        raise AssertionError("n_raw >= 2^31 accepted")
    g = oracle.build_graph([3], np.array([np.nan, 2.0, np.inf], np.float32), lib_path=lib)
    r, it, res = g.pagerank(0.85, 1e-13, MAX_ITER)
    assert g.N == 1 and g.M == 1 and r[0] == 1.0 and g.score(r, 0.0)[0] == 1.0
    for d in (0.0, 1.0, -0.5, 1.5, float("nan")):
        try:
            g.pagerank(d)
        except oracle.OracleError as e:
            assert e.code == oracle.EINVAL
        else:
            raise AssertionError(f"damping {d} accepted")


QUICK = [check_paper_sizes, check_adjacent_example, check_neighbours_product_order,
         check_ffg_bruteforce, check_pagerank_dense, check_closed_forms,
         check_separable_minima, check_plateau_minima, check_naive_separable, check_score_brute,
         check_dag_rank, check_metamorphic, check_errors]


def run_quick(lib):
    """Run every quick check; return the names of those that failed."""
    failed = []
    for chk in QUICK:
        try:
            chk(lib)
        except (AssertionError, oracle.OracleError):
            failed.append(chk.__name__)
    return failed
