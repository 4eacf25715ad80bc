"""FP64 CPU oracle for the fitness-flow-graph landscape metric.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  The GPU engine never does, and it
shares no code with it.

This module is a thin ctypes wrapper over ``flo.c`` (plain C, FP64,
single-threaded), which follows the paper's definitions: search space and
neighbourhoods (Sec. III-B, eq. 2), failed configurations (Sec. V), fitness
flow graph, PageRank centrality and the p-proportion of centrality
(Sec. VII-B, eq. 3), and the naive metric f_opt / f over the local minima
(Sec. VII-A).  ``build()`` compiles it with gcc.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "flo.c")
LIB = os.path.join(HERE, "liboracle.so")

HAMMING, ADJACENT = 0, 1
OK, EINVAL, ENOMEM, ENOCONV, EOVERFLOW = 0, -1, -2, -4, -5


def build(src: str = SRC, out: str = LIB, extra: tuple = ()) -> str:
    """Compile the oracle into a shared library (always recompiles)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           *extra, "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_lib_cache: dict = {}


def load(path: str = LIB) -> ctypes.CDLL:
    """Load a built oracle library (building it only if nothing is built)."""
    if path in _lib_cache:
        return _lib_cache[path]
    if not os.path.exists(path):
        build(out=path)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.flo_build.argtypes = [ctypes.c_int, P, P, ctypes.c_int, ctypes.POINTER(P)]
    lib.flo_build.restype = ctypes.c_int
    lib.flo_free.argtypes = [P]
    lib.flo_free.restype = None
    lib.flo_sizes.argtypes = [P, i64p]
    lib.flo_sizes.restype = None
    lib.flo_f_opt.argtypes = [P]
    lib.flo_f_opt.restype = ctypes.c_double
    lib.flo_export.argtypes = [P, P, P, P, P, P, P]
    lib.flo_export.restype = None
    lib.flo_neighbour_list.argtypes = [P, ctypes.c_int64, P]
    lib.flo_neighbour_list.restype = ctypes.c_int64
    lib.flo_pagerank.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                 P, i64p, ctypes.POINTER(ctypes.c_double)]
    lib.flo_pagerank.restype = ctypes.c_int
    lib.flo_score.argtypes = [P, P, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double)]
    lib.flo_score.restype = ctypes.c_double
    lib.flo_dag_rank.argtypes = [P, ctypes.c_double, P, i64p]
    lib.flo_dag_rank.restype = ctypes.c_int
    lib.flo_naive.argtypes = [P, P, ctypes.c_int64, P]
    lib.flo_naive.restype = ctypes.c_int
    lib.flo_analyze.argtypes = [ctypes.c_int, P, P, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int64, P, P, P, P, P, ctypes.c_int64, P, P]
    lib.flo_analyze.restype = ctypes.c_int
    _lib_cache[path] = lib
    return lib


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with status {code}")
        self.code = code


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


@dataclass
class Graph:
    """The FFG of one space, as computed by the oracle."""
    radix: tuple
    n_raw: int
    N: int
    E: int
    M: int
    plateau_minima: int
    K: int
    f_opt: float
    valid_raw: np.ndarray   # int32[N]  node id -> raw index
    row_ptr: np.ndarray     # int32[N+1] CSR over in-edges
    col_idx: np.ndarray     # int32[E]  sources, ascending per row
    out_deg: np.ndarray     # int32[N]
    minima: np.ndarray      # int32[M]  ascending node ids
    fit: np.ndarray         # float32[N]
    _handle: ctypes.c_void_p = None
    _lib: ctypes.CDLL = None

    def neighbours(self, v: int) -> np.ndarray:
        """Raw indices of the valid neighbours of node v (sorted)."""
        out = np.empty(int(sum(self.radix)), dtype=np.int32)
        k = self._lib.flo_neighbour_list(self._handle, int(v), _ptr(out))
        if k < 0:
            raise OracleError(int(k), "flo_neighbour_list")
        return np.sort(out[:k])

    def pagerank(self, damping: float = 0.85, tol: float = 1e-13,
                 max_iter: int = 1_000_000, check: bool = True):
        r = np.empty(self.N, dtype=np.float64)
        it = ctypes.c_int64()
        res = ctypes.c_double()
        rc = self._lib.flo_pagerank(self._handle, damping, tol, max_iter, _ptr(r),
                                    ctypes.byref(it), ctypes.byref(res))
        if rc not in (OK, ENOCONV) or (check and rc != OK):
            raise OracleError(rc, "flo_pagerank")
        return r, int(it.value), float(res.value)

    def dag_rank(self, damping: float = 0.85):
        """Exact PageRank by forward substitution in descending fitness order
        (valid for damping in (0, 1]); returns (r, longest path length)."""
        r = np.empty(self.N, dtype=np.float64)
        depth = ctypes.c_int64()
        rc = self._lib.flo_dag_rank(self._handle, damping, _ptr(r), ctypes.byref(depth))
        if rc != 0:
            raise OracleError(rc, "flo_dag_rank")
        return r, int(depth.value)

    def score(self, centrality: np.ndarray, p: float):
        c = np.ascontiguousarray(centrality, dtype=np.float64)
        num, den = ctypes.c_double(), ctypes.c_double()
        s = self._lib.flo_score(self._handle, _ptr(c), p, ctypes.byref(num), ctypes.byref(den))
        return float(s), float(num.value), float(den.value)

    def naive(self, n_bins: int = 20):
        """Naive metric (flo_naive): f_opt / f(m) for every local minimum in
        ascending node id (float64[M]) and its histogram over n_bins equal
        bins of [0, 1] (int64[n_bins])."""
        ratio = np.empty(max(self.M, 1), dtype=np.float64)
        hist = np.empty(max(int(n_bins), 1), dtype=np.int64)
        rc = self._lib.flo_naive(self._handle, _ptr(ratio), int(n_bins), _ptr(hist))
        if rc != OK:
            raise OracleError(rc, "flo_naive")
        return ratio[:self.M], hist[:int(n_bins)]

    def close(self):
        if self._handle:
            self._lib.flo_free(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_graph(radix, fitness_raw, neighbourhood: int = HAMMING,
                lib_path: str = LIB) -> Graph:
    """Build the FFG of a space (raises OracleError on an invalid input)."""
    lib = load(lib_path)
    rad = np.ascontiguousarray(radix, dtype=np.int32)
    fit = np.ascontiguousarray(fitness_raw, dtype=np.float32)
    h = ctypes.c_void_p()
    rc = lib.flo_build(len(rad), _ptr(rad), _ptr(fit), int(neighbourhood), ctypes.byref(h))
    if rc != OK:
        raise OracleError(rc, "flo_build")
    sizes = np.zeros(6, dtype=np.int64)
    lib.flo_sizes(h, sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    n_raw, N, E, M, plateau, K = (int(s) for s in sizes)
    valid_raw = np.empty(N, np.int32)
    row_ptr = np.empty(N + 1, np.int32)
    col_idx = np.empty(max(E, 1), np.int32)
    out_deg = np.empty(N, np.int32)
    minima = np.empty(max(M, 1), np.int32)
    f = np.empty(N, np.float32)
    lib.flo_export(h, _ptr(valid_raw), _ptr(row_ptr), _ptr(col_idx), _ptr(out_deg),
                   _ptr(minima), _ptr(f))
    return Graph(tuple(int(r) for r in rad), n_raw, N, E, M, plateau, K, float(lib.flo_f_opt(h)), valid_raw,
                 row_ptr, col_idx[:E], out_deg, minima[:M], f, h, lib)


@dataclass
class Analysis:
    graph: Graph
    pagerank: np.ndarray
    iterations: int
    residual: float
    score: float
    mass_near: float
    mass_minima: float


def analyze(radix, fitness_raw, neighbourhood: int = HAMMING, damping: float = 0.85,
            p: float = 0.05, tol: float = 1e-13, max_iter: int = 1_000_000,
            lib_path: str = LIB) -> Analysis:
    """FFG + PageRank + C_p of one space, all on the oracle."""
    g = build_graph(radix, fitness_raw, neighbourhood, lib_path)
    r, it, res = g.pagerank(damping, tol, max_iter)
    s, num, den = g.score(r, p)
    return Analysis(g, r, it, res, s, num, den)


ESIZE = -6


def analyze_one_call(radix, fitness_raw, neighbourhood: int = HAMMING, damping: float = 0.85,
                     p: float = 0.05, tol: float = 1e-13, max_iter: int = 1_000_000,
                     cap_edges: int | None = None, lib_path: str = LIB) -> dict:
    """The whole analysis through the library's one-call entry point
    (flo_analyze); host buffers sized from n_raw, col_idx from cap_edges
    (default: the candidate-pair bound n_raw * K).  Returns the status and
    every output; arrays are cut to their sizes when the call succeeded."""
    lib = load(lib_path)
    rad = np.ascontiguousarray(radix, dtype=np.int32)
    fit = np.ascontiguousarray(fitness_raw, dtype=np.float32)
    n_raw = int(np.prod(rad.astype(np.int64)))
    K = int(sum((min(int(r) - 1, 2) if neighbourhood == ADJACENT else int(r) - 1) for r in rad))
    cap = n_raw * max(K, 1) if cap_edges is None else int(cap_edges)
    pr = np.zeros(max(n_raw, 1), np.float64)
    minima = np.zeros(max(n_raw, 1), np.int32)
    valid_raw = np.zeros(max(n_raw, 1), np.int32)
    row_ptr = np.zeros(n_raw + 1, np.int32)
    col_idx = np.zeros(max(cap, 1), np.int32)
    sizes = np.zeros(7, np.int64)
    stats = np.zeros(5, np.float64)
    rc = lib.flo_analyze(len(rad), _ptr(rad), _ptr(fit), int(neighbourhood), float(damping), float(p), float(tol),
                         int(max_iter), _ptr(pr), _ptr(minima), _ptr(valid_raw), _ptr(row_ptr), _ptr(col_idx),
                         cap, _ptr(sizes), _ptr(stats))
    n_raw_, N, E, M, plateau, iters, K_ = (int(v) for v in sizes)
    out = {"status": int(rc), "n_raw": n_raw_, "N": N, "E": E, "M": M, "plateau_minima": plateau,
           "iterations": iters, "K": K_}
    if rc in (OK, ENOCONV):
        out.update(pagerank=pr[:N], minima=minima[:M], valid_raw=valid_raw[:N], row_ptr=row_ptr[:N + 1],
                   col_idx=col_idx[:E], residual=float(stats[0]), f_opt=float(stats[1]), score=float(stats[2]),
                   mass_near=float(stats[3]), mass_minima=float(stats[4]))
    return out
