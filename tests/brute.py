"""Brute-force and closed-form references used to pin the oracle.

Nothing here shares code with ``oracle/flo.c``; each routine reaches the same
quantity by a different route:

* configurations are enumerated with ``itertools.product`` and neighbours are
  found by comparing digit tuples of all pairs (no stride arithmetic);
* the FFG is rebuilt from those pairs;
* PageRank is a dense linear solve, or the dense eigenvector for eigenvalue 1;
* an exact DAG identity gives PageRank at any size (see ``dag_pagerank``);
* a vectorised per-axis grid comparison gives degrees and edge counts at any
  size (see ``grid_degrees``).

Pure-Python loops are used only on small inputs.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def configs(radix):
    """Digit tuples in raw order (parameter 0 most significant)."""
    return list(itertools.product(*[range(int(r)) for r in radix]))


def is_valid(v: float) -> bool:
    return bool(np.isfinite(v) and v > 0)


def are_neighbours(x, y, neighbourhood: str) -> bool:
    """Sec. III-B: differ in exactly one coordinate; for 'adjacent' that
    coordinate's list positions must be next to each other."""
    diff = [i for i in range(len(x)) if x[i] != y[i]]
    if len(diff) != 1:
        return False
    if neighbourhood == "adjacent":
        i = diff[0]
        return abs(x[i] - y[i]) == 1
    return True


class BruteFFG:
    """FFG of a small space by all-pairs comparison of digit tuples."""

    def __init__(self, radix, fitness_raw, neighbourhood: str = "hamming"):
        cfg = configs(radix)
        f = np.asarray(fitness_raw, dtype=np.float32)
        assert len(cfg) == f.size
        self.raw = [i for i in range(len(cfg)) if is_valid(f[i])]
        self.N = len(self.raw)
        self.f = np.array([f[i] for i in self.raw], dtype=np.float32)
        digits = [cfg[i] for i in self.raw]
        self.nbrs = [[] for _ in range(self.N)]
        for a in range(self.N):
            for b in range(self.N):
                if a != b and are_neighbours(digits[a], digits[b], neighbourhood):
                    self.nbrs[a].append(b)
        # edge a -> b iff b is a neighbour with strictly lower fitness
        self.out = [[b for b in self.nbrs[a] if self.f[b] < self.f[a]] for a in range(self.N)]
        self.inn = [[] for _ in range(self.N)]
        for a in range(self.N):
            for b in self.out[a]:
                self.inn[b].append(a)
        self.inn = [sorted(lst) for lst in self.inn]
        self.out_deg = np.array([len(o) for o in self.out], dtype=np.int64)
        self.E = int(self.out_deg.sum())
        self.minima = [v for v in range(self.N)
                       if all(self.f[w] >= self.f[v] for w in self.nbrs[v])]
        self.f_opt = float(self.f.min())

    def csr(self):
        row_ptr = np.zeros(self.N + 1, dtype=np.int64)
        for v in range(self.N):
            row_ptr[v + 1] = row_ptr[v] + len(self.inn[v])
        col = np.array([u for v in range(self.N) for u in self.inn[v]], dtype=np.int64)
        return row_ptr, col

    def google_matrix(self, d: float) -> np.ndarray:
        """G = d (P + 1 s^T / N) + (1-d)/N 1 1^T, column-stochastic."""
        N = self.N
        B = np.zeros((N, N))
        for u in range(N):
            if self.out_deg[u] == 0:
                B[:, u] = 1.0 / N
            else:
                for w in self.out[u]:
                    B[w, u] = 1.0 / self.out_deg[u]
        return d * B + (1.0 - d) / N * np.ones((N, N))

    def pagerank_solve(self, d: float) -> np.ndarray:
        """r with G r = r, sum r = 1, via (I - d B) r = (1-d)/N 1."""
        N = self.N
        G = self.google_matrix(d)
        B = (G - (1.0 - d) / N) / d
        r = np.linalg.solve(np.eye(N) - d * B, np.full(N, (1.0 - d) / N))
        return r / r.sum()

    def pagerank_eig(self, d: float) -> np.ndarray:
        w, V = np.linalg.eig(self.google_matrix(d))
        k = int(np.argmin(np.abs(w - 1.0)))
        r = np.real(V[:, k])
        return r / r.sum()


def dag_pagerank(N: int, row_ptr, col_idx, out_deg, d: float) -> np.ndarray:
    """Exact PageRank of a DAG with uniform teleport and uniform sink spreading.

    G r = r expands to r = d P r + beta 1 with a scalar beta, because both the
    teleport and the sink term are multiples of the all-ones vector.  Hence
    r = u / sum(u) with (I - d P) u = 1.  P is nilpotent on a DAG, so the
    Jacobi sweep u <- 1 + d P u reaches u exactly after (longest path + 1)
    sweeps and then stops changing bit for bit.  No power iteration, no
    teleport bookkeeping and no sink handling is involved.
    """
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    deg = np.asarray(out_deg, dtype=np.float64)
    rows = np.repeat(np.arange(N), np.diff(row_ptr))
    vals = 1.0 / deg[col_idx] if col_idx.size else np.zeros(0)
    P = sp.csr_matrix((vals, (rows, col_idx)), shape=(N, N))
    u = np.ones(N)
    for _ in range(N + 1):
        nu = 1.0 + d * (P @ u)
        if np.array_equal(nu, u):
            return u / u.sum()
        u = nu
    raise AssertionError("DAG sweep did not settle: the graph has a cycle")


def grid_degrees(radix, fitness_raw, neighbourhood: str = "hamming"):
    """In/out degree of every raw configuration by whole-array comparisons.

    For every axis i and every ordered pair of list positions (a, b) that are
    neighbours along that axis, the slices f[..., a, ...] and f[..., b, ...]
    are compared elementwise (numpy indexing, no stride arithmetic).
    Returns (in_deg, out_deg, valid) as arrays of shape ``radix``; degrees of
    invalid configurations are 0.
    """
    f = np.asarray(fitness_raw, dtype=np.float32).reshape(tuple(radix))
    valid = np.isfinite(f) & (f > 0)
    fv = np.where(valid, f, np.float32(np.nan))  # NaN compares false
    in_deg = np.zeros(f.shape, dtype=np.int64)
    out_deg = np.zeros(f.shape, dtype=np.int64)
    for i, r in enumerate(radix):
        for a in range(r):
            for b in range(r):
                if a == b or (neighbourhood == "adjacent" and abs(a - b) != 1):
                    continue
                ia = [slice(None)] * len(radix)
                ib = [slice(None)] * len(radix)
                ia[i], ib[i] = a, b
                fa, fb = fv[tuple(ia)], fv[tuple(ib)]
                out_deg[tuple(ia)] += (fb < fa)   # b is a better neighbour of a
                in_deg[tuple(ia)] += (fb > fa)    # b flows into a
    return in_deg, out_deg, valid


def kahn_acyclic(N: int, row_ptr, col_idx) -> bool:
    """Kahn's algorithm on the in-edge CSR: True iff the graph has no cycle."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    indeg = np.diff(row_ptr).copy()
    outs = [[] for _ in range(N)]
    for w in range(N):
        for e in range(row_ptr[w], row_ptr[w + 1]):
            outs[col_idx[e]].append(w)
    stack = [v for v in range(N) if indeg[v] == 0]
    seen = 0
    while stack:
        u = stack.pop()
        seen += 1
        for w in outs[u]:
            indeg[w] -= 1
            if indeg[w] == 0:
                stack.append(w)
    return seen == N
