"""Python binding of the C ABI (include/fl.h): argument marshalling only.

Every step of the analysis runs in the HIP kernels of ``libfl.so``; torch
provides device memory and the stream.  Function names follow the C entry
points without the ``fl_`` prefix:

    create / destroy / last_error      fl_create / fl_destroy / fl_last_error
    plan_create                        fl_plan_create   (build the FFG)
    execute                            fl_execute       (PageRank, minima, C_p)
    execute(exact=True)                fl_execute_exact (exact sweeps, damping in (0, 1])
    plan_export / plan_timing          fl_plan_export / fl_plan_timing
    tune                               fl_tune          (autotune the sweep layout)
    profile                            fl_profile       (per-sweep device timing)
    score_curve                        fl_score_curve   (C_p for many p)
    naive_metric                       fl_naive_metric  (f_opt / f over the minima)
    plan_destroy                       fl_plan_destroy
    analyze                            fl_analyze       (one shot)
    analyze(no_alloc=True)             fl_analyze_noalloc (one shot, no device allocation)
    Batch / batch_create               fl_batch_create / _add / _step / _collect / _timing / _destroy
    analyze_batch                      fl_analyze_batch (many spaces, one shot)
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _abi

NEIGHBOURHOODS = {"hamming": _abi.FL_NB_HAMMING, "adjacent": _abi.FL_NB_ADJACENT}


class FLError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: {_abi.STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.message = message


def _check(ctx, status: int, where: str, allow=()):
    if status != _abi.FL_OK and status not in allow:
        msg = _abi.load().fl_last_error(ctx.handle if ctx else None).decode(errors="replace")
        raise FLError(status, where, msg)
    return status


def _nb(neighbourhood) -> int:
    if isinstance(neighbourhood, str):
        return NEIGHBOURHOODS[neighbourhood]
    return int(neighbourhood)


def _space(radix):
    arr = (ctypes.c_int32 * len(radix))(*[int(r) for r in radix])
    sp = _abi.fl_space(len(radix), ctypes.cast(arr, ctypes.POINTER(ctypes.c_int32)))
    return sp, arr


def _n_raw(radix) -> int:
    n = 1
    for r in radix:
        n *= int(r)
    return n


def _check_fitness(ctx: "Context", radix, fitness_raw: torch.Tensor):
    # the kernels read prod(radix) floats: the tensor must hold exactly that
    if not isinstance(fitness_raw, torch.Tensor):
        raise TypeError("fitness_raw must be a torch tensor")
    if fitness_raw.dtype != torch.float32 or not fitness_raw.is_cuda:
        raise TypeError("fitness_raw must be a float32 tensor on the GPU")
    if fitness_raw.device.index != ctx.device:
        raise ValueError(f"fitness_raw is on {fitness_raw.device}, context on cuda:{ctx.device}")
    if not fitness_raw.is_contiguous() or fitness_raw.numel() != _n_raw(radix):
        raise ValueError(f"fitness_raw must be contiguous with prod(radix) = {_n_raw(radix)} "
                         f"entries, got {fitness_raw.numel()}")


class Context:
    """An ``fl_ctx`` bound to a device and a torch stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        lib = _abi.load()
        self.device = int(device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.handle = ctypes.c_void_p()
        rc = lib.fl_create(ctypes.byref(self.handle), self.device,
                           ctypes.c_void_p(self.stream.cuda_stream))
        if rc != _abi.FL_OK:
            raise FLError(rc, "fl_create", f"device {self.device}")

    def close(self):
        if self.handle:
            _abi.load().fl_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def create(device: int = 0, stream=None) -> Context:
    return Context(device, stream)


def destroy(ctx: Context) -> None:
    ctx.close()


def last_error(ctx: Context) -> str:
    return _abi.load().fl_last_error(ctx.handle).decode(errors="replace")


@dataclass
class Plan:
    ctx: Context
    handle: ctypes.c_void_p
    radix: tuple
    sizes: dict

    @property
    def n_valid(self) -> int:
        return int(self.sizes["n_valid"])

    @property
    def n_edges(self) -> int:
        return int(self.sizes["n_edges"])

    @property
    def n_minima(self) -> int:
        return int(self.sizes["n_minima"])

    def close(self):
        if self.handle:
            _abi.load().fl_plan_destroy(self.ctx.handle, self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_create(ctx: Context, radix, fitness_raw: torch.Tensor, neighbourhood="hamming") -> Plan:
    """Build the FFG of one space (fl_plan_create)."""
    _check_fitness(ctx, radix, fitness_raw)
    sp, keep = _space(radix)
    h = ctypes.c_void_p()
    sizes = _abi.fl_summary()
    rc = _abi.load().fl_plan_create(ctx.handle, ctypes.byref(sp),
                                    ctypes.c_void_p(fitness_raw.data_ptr()), _nb(neighbourhood),
                                    ctypes.byref(h), ctypes.byref(sizes))
    _check(ctx, rc, "fl_plan_create")
    del keep
    return Plan(ctx, h, tuple(int(r) for r in radix), sizes.as_dict())


def _params(damping, p, tol, max_iter, row_mapping, separate_step=False):
    return _abi.fl_params(float(damping), float(p), float(tol), int(max_iter), int(row_mapping),
                          _abi.FL_STEP_SEPARATE if separate_step else 0, 0)


def execute(plan: Plan, damping: float = 0.85, p: float = 0.05, tol: float = 0.0,
            max_iter: int = 0, row_mapping: int = 0, pagerank: torch.Tensor | None = None,
            minima: torch.Tensor | None = None, allow_noconv: bool = False, exact: bool = False,
            separate_step: bool = False):
    """PageRank, local minima and C_p on a plan (fl_execute; with exact=True
    fl_execute_exact, which also accepts damping 1).  separate_step=True
    (FL_STEP_SEPARATE) runs a step kernel after every sweep, the order of
    sums a batch uses, instead of the lagged step.

    Returns (pagerank float64[N], minima int32[M], summary dict).  Output
    tensors may be passed in (sizes N and M, on the context's device)."""
    ctx = plan.ctx
    dev = torch.device("cuda", ctx.device)
    if pagerank is None:
        pagerank = torch.empty(plan.n_valid, dtype=torch.float64, device=dev)
    if minima is None:
        minima = torch.empty(max(plan.n_minima, 1), dtype=torch.int32, device=dev)
    if (pagerank.dtype != torch.float64 or pagerank.numel() < plan.n_valid
            or not pagerank.is_contiguous() or pagerank.device != dev):
        raise ValueError("pagerank must be a contiguous float64 tensor of >= N entries")
    if (minima.dtype != torch.int32 or minima.numel() < plan.n_minima
            or not minima.is_contiguous() or minima.device != dev):
        raise ValueError("minima must be a contiguous int32 tensor of >= M entries")
    prm = _params(damping, p, tol, max_iter, row_mapping, separate_step)
    out = _abi.fl_summary()
    fn = _abi.load().fl_execute_exact if exact else _abi.load().fl_execute
    rc = fn(ctx.handle, plan.handle, ctypes.byref(prm), ctypes.c_void_p(pagerank.data_ptr()),
            ctypes.c_void_p(minima.data_ptr()), ctypes.byref(out))
    _check(ctx, rc, "fl_execute_exact" if exact else "fl_execute",
           allow=(_abi.FL_ENOCONV,) if allow_noconv else ())
    info = out.as_dict()
    info["status"] = rc
    return pagerank[:plan.n_valid], minima[:plan.n_minima], info


def plan_export(plan: Plan) -> dict:
    """The plan's FFG as device tensors (fl_plan_export)."""
    ctx = plan.ctx
    dev = torch.device("cuda", ctx.device)
    N, E = plan.n_valid, plan.n_edges
    t = {"valid_raw": torch.empty(N, dtype=torch.int32, device=dev),
         "row_ptr": torch.empty(N + 1, dtype=torch.int32, device=dev),
         "col_idx": torch.empty(max(E, 1), dtype=torch.int32, device=dev),
         "out_deg": torch.empty(N, dtype=torch.int32, device=dev)}
    rc = _abi.load().fl_plan_export(ctx.handle, plan.handle,
                                    *[ctypes.c_void_p(t[k].data_ptr())
                                      for k in ("valid_raw", "row_ptr", "col_idx", "out_deg")])
    _check(ctx, rc, "fl_plan_export")
    t["col_idx"] = t["col_idx"][:E]
    return t


ROWS_SLOTS = -1
ROWS_BINNED = -2
TUNE_LAYOUTS = (ROWS_SLOTS, 1, 2, 4, 8, 16, 32, 64, ROWS_BINNED)


def tune(plan: Plan, damping: float = 0.85, sweeps: int = 4) -> dict:
    """Autotune the in-degree bucket mapping and the sweep layout for the
    plan's shape class (fl_tune).  Returns {"best": layout, "us_per_sweep":
    {layout: us}, "buckets": bucket_map(plan)} (-1 slot sweep, -2 binned
    sweep, else CSR lanes per row)."""
    best = ctypes.c_int32()
    times = (ctypes.c_double * len(TUNE_LAYOUTS))()
    prm = _params(damping, 0.05, 0.0, 0, 0)
    rc = _abi.load().fl_tune(plan.ctx.handle, plan.handle, ctypes.byref(prm), int(sweeps),
                             ctypes.byref(best), times)
    _check(plan.ctx, rc, "fl_tune")
    return {"best": int(best.value),
            "us_per_sweep": {lay: float(t) for lay, t in zip(TUNE_LAYOUTS, times) if t >= 0},
            "buckets": bucket_map(plan)}


BUCKETS = ("0", "1", "2-3", "4-7", "8-15", "16-31", "32-63", "64+")


def bucket_map(plan: Plan) -> dict:
    """The context's in-degree bucket mapping for the plan's shape class and
    the plan's rows per bucket (fl_bucket_map): {bucket: {"lanes", "blocks",
    "rows"}} with buckets named by their in-degree range."""
    lanes = (ctypes.c_int32 * 8)()
    blocks = (ctypes.c_int32 * 8)()
    rows = (ctypes.c_int64 * 8)()
    rc = _abi.load().fl_bucket_map(plan.ctx.handle, plan.handle, lanes, blocks, rows)
    _check(plan.ctx, rc, "fl_bucket_map")
    return {BUCKETS[b]: {"lanes": int(lanes[b]), "blocks": int(blocks[b]), "rows": int(rows[b])} for b in range(8)}


def score_curve(plan: Plan, pagerank: torch.Tensor, p_values=tuple(j / 100 for j in range(16))) -> list:
    """C_p for every proportion in p_values (fl_score_curve), from the ranks
    that execute() returned for this plan.  Default: p = 0, 1, ..., 15 %."""
    ps = [float(x) for x in p_values]
    n = len(ps)
    if pagerank.dtype != torch.float64 or pagerank.numel() < plan.n_valid or not pagerank.is_cuda:
        raise ValueError("pagerank must be the float64 device tensor execute() returned")
    pa = (ctypes.c_double * max(n, 1))(*ps)
    out = (ctypes.c_double * max(n, 1))()
    rc = _abi.load().fl_score_curve(plan.ctx.handle, plan.handle, ctypes.c_void_p(pagerank.data_ptr()), n, pa, out)
    _check(plan.ctx, rc, "fl_score_curve")
    return [float(out[j]) for j in range(n)]


def naive_metric(plan: Plan, n_bins: int = 20):
    """f_opt / f(m) for every local minimum (device float64 tensor, ascending
    node id) and its histogram over n_bins equal bins of [0, 1] (fl_naive_metric)."""
    dev = torch.device("cuda", plan.ctx.device)
    ratio = torch.empty(max(plan.n_minima, 1), dtype=torch.float64, device=dev)
    hist = (ctypes.c_int64 * max(int(n_bins), 1))()
    rc = _abi.load().fl_naive_metric(plan.ctx.handle, plan.handle, ctypes.c_void_p(ratio.data_ptr()),
                                     int(n_bins), hist)
    _check(plan.ctx, rc, "fl_naive_metric")
    return ratio[:plan.n_minima], [int(hist[j]) for j in range(int(n_bins))]


def profile(ctx: Context, every: int = 1) -> None:
    """Time every every-th sweep kernel with HIP events (fl_profile; 0 = off);
    see plan_timing's sweep_ms and sweeps_timed."""
    _check(ctx, _abi.load().fl_profile(ctx.handle, int(every)), "fl_profile")


def plan_timing(plan: Plan) -> dict:
    out = _abi.fl_timing()
    rc = _abi.load().fl_plan_timing(plan.ctx.handle, plan.handle, ctypes.byref(out))
    _check(plan.ctx, rc, "fl_plan_timing")
    return out.as_dict()


def plan_destroy(plan: Plan) -> None:
    plan.close()


@dataclass
class Result:
    pagerank: torch.Tensor   # float64[N]
    minima: torch.Tensor     # int32[M], ascending node ids
    valid_raw: torch.Tensor  # int32[N], node id -> raw index
    score: float
    info: dict


def analyze(radix, fitness_raw: torch.Tensor, neighbourhood="hamming", damping: float = 0.85,
            p: float = 0.05, tol: float = 0.0, max_iter: int = 0, row_mapping: int = 0,
            ctx: Context | None = None, allow_noconv: bool = False, no_alloc: bool = False,
            out: tuple | None = None) -> Result:
    """One-shot analysis of one space (fl_analyze; with no_alloc=True
    fl_analyze_noalloc, whose device buffers all live in the library's fixed
    scratch array).  ``out`` may pass the three output tensors
    (pagerank float64, minima int32, valid_raw int32, each >= prod(radix)
    entries on the context's device); otherwise they are allocated here."""
    own = ctx is None
    if own:
        ctx = Context(fitness_raw.device.index or 0)
    try:
        _check_fitness(ctx, radix, fitness_raw)
        n_raw = _n_raw(radix)
        dev = fitness_raw.device
        if out is None:
            pr = torch.empty(n_raw, dtype=torch.float64, device=dev)
            mins = torch.empty(n_raw, dtype=torch.int32, device=dev)
            vraw = torch.empty(n_raw, dtype=torch.int32, device=dev)
        else:
            pr, mins, vraw = out
            for t, dt in ((pr, torch.float64), (mins, torch.int32), (vraw, torch.int32)):
                if t.dtype != dt or t.numel() < n_raw or not t.is_contiguous() or t.device != dev:
                    raise ValueError("out tensors must be contiguous (float64, int32, int32) with "
                                     f">= {n_raw} entries on {dev}")
        sp, keep = _space(radix)
        prm = _params(damping, p, tol, max_iter, row_mapping)
        summ = _abi.fl_summary()
        name = "fl_analyze_noalloc" if no_alloc else "fl_analyze"
        rc = getattr(_abi.load(), name)(ctx.handle, ctypes.byref(sp),
                                        ctypes.c_void_p(fitness_raw.data_ptr()), _nb(neighbourhood),
                                        ctypes.byref(prm), ctypes.c_void_p(pr.data_ptr()),
                                        ctypes.c_void_p(mins.data_ptr()),
                                        ctypes.c_void_p(vraw.data_ptr()), ctypes.byref(summ))
        _check(ctx, rc, name, allow=(_abi.FL_ENOCONV,) if allow_noconv else ())
        del keep
        info = summ.as_dict()
        info["status"] = rc
        N, M = int(summ.n_valid), int(summ.n_minima)
        return Result(pr[:N], mins[:M], vraw[:N], float(summ.score), info)
    finally:
        if own:
            ctx.close()


class Batch:
    """An ``fl_batch``: plans swept together (fl_batch_* entry points).

    ``add`` attaches a plan with its parameters and output tensors, ``step``
    runs sweeps for all running members, ``collect`` returns the finished
    ones as ``(tag, pagerank, minima, summary)``.
    """

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self.handle = ctypes.c_void_p()
        _check(ctx, _abi.load().fl_batch_create(ctx.handle, ctypes.byref(self.handle)), "fl_batch_create")
        self._outputs = {}
        self._next_tag = 0

    def add(self, plan: Plan, damping: float = 0.85, p: float = 0.05, tol: float = 0.0,
            max_iter: int = 0, tag: int | None = None, row_mapping: int = 0) -> int:
        """Add a member; returns its tag.  Without a tag the next unused one
        of an increasing counter is taken.  A tag of a member that has not
        been collected yet is rejected (ValueError): its output tensors are
        still being written.  row_mapping: 0 (automatic), ROWS_SLOTS or
        ROWS_BINNED."""
        if tag is None:
            while self._next_tag in self._outputs:
                self._next_tag += 1
            tag = self._next_tag
            self._next_tag += 1
        else:
            tag = int(tag)
        if tag in self._outputs:
            raise ValueError(f"tag {tag} belongs to a member that has not been collected")
        dev = torch.device("cuda", self.ctx.device)
        pr = torch.empty(plan.n_valid, dtype=torch.float64, device=dev)
        mins = torch.empty(max(plan.n_minima, 1), dtype=torch.int32, device=dev)
        prm = _params(damping, p, tol, max_iter, row_mapping)
        rc = _abi.load().fl_batch_add(self.ctx.handle, self.handle, plan.handle, ctypes.byref(prm),
                                      ctypes.c_void_p(pr.data_ptr()), ctypes.c_void_p(mins.data_ptr()), tag)
        _check(self.ctx, rc, "fl_batch_add")
        self._outputs[tag] = (plan, pr, mins)
        return tag

    def step(self, sweeps: int = 8) -> int:
        running = ctypes.c_int32()
        rc = _abi.load().fl_batch_step(self.ctx.handle, self.handle, int(sweeps), ctypes.byref(running))
        _check(self.ctx, rc, "fl_batch_step")
        return int(running.value)

    def collect(self, max_items: int = 1024) -> list:
        tags = (ctypes.c_int64 * max_items)()
        sums = (_abi.fl_summary * max_items)()
        n = ctypes.c_int32()
        rc = _abi.load().fl_batch_collect(self.ctx.handle, self.handle, max_items, tags, sums, ctypes.byref(n))
        _check(self.ctx, rc, "fl_batch_collect")
        out = []
        for j in range(n.value):
            plan, pr, mins = self._outputs.pop(int(tags[j]))
            info = sums[j].as_dict()
            out.append((int(tags[j]), pr, mins[:plan.n_minima], info))
        return out

    def timing(self) -> dict:
        sweeps, launches, captures = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        ms = ctypes.c_double()
        _check(self.ctx, _abi.load().fl_batch_timing(self.ctx.handle, self.handle, ctypes.byref(sweeps),
                                                      ctypes.byref(ms), ctypes.byref(launches),
                                                      ctypes.byref(captures)), "fl_batch_timing")
        return {"sweeps": int(sweeps.value), "sweep_ms": float(ms.value),
                "graph_launches": int(launches.value), "graph_captures": int(captures.value)}

    def set_graphs(self, enable: bool) -> None:
        """Replay the captured sweep loop (default) or launch kernel by kernel."""
        _check(self.ctx, _abi.load().fl_batch_set_graphs(self.ctx.handle, self.handle, int(bool(enable))),
               "fl_batch_set_graphs")

    def set_small(self, max_tiles: int) -> None:
        """Members of at most max_tiles tiles of 256 nodes iterate in one
        workgroup each (fl_batch_set_small; 0 = none, default 16)."""
        _check(self.ctx, _abi.load().fl_batch_set_small(self.ctx.handle, self.handle, int(max_tiles)),
               "fl_batch_set_small")

    def close(self):
        if self.handle:
            _abi.load().fl_batch_destroy(self.ctx.handle, self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_create(ctx: Context) -> Batch:
    return Batch(ctx)


def analyze_batch(spaces, fitness, neighbourhood="hamming", damping=0.85, p: float = 0.05,
                  tol: float = 0.0, max_iter: int = 0, ctx: Context | None = None) -> list:
    """fl_analyze_batch over many spaces.  ``spaces`` is a list of radix
    tuples, ``fitness`` a matching list of device float32 tensors on the
    context's device; the other arguments may be scalars or per-space lists.
    Returns a list of Result whose pagerank and minima tensors are views into
    one float64 and one int32 buffer shared by the call's results."""
    n = len(spaces)
    if len(fitness) != n:
        raise ValueError("spaces and fitness differ in length")
    own = ctx is None
    if own:
        ctx = Context(fitness[0].device.index or 0 if n else 0)

    def per(x):
        return list(x) if isinstance(x, (list, tuple)) else [x] * n
    nbs, ds, ps, tols, its = per(neighbourhood), per(damping), per(p), per(tol), per(max_iter)
    try:
        keep = []
        sp_arr = (_abi.fl_space * max(n, 1))()
        fit_ptrs = (ctypes.c_void_p * max(n, 1))()
        nb_arr = (ctypes.c_int * max(n, 1))()
        prm_arr = (_abi.fl_params * max(n, 1))()
        pr_ptrs = (ctypes.c_void_p * max(n, 1))()
        min_ptrs = (ctypes.c_void_p * max(n, 1))()
        outs = (_abi.fl_summary * max(n, 1))()
        # one output buffer per type for all spaces: space j owns n_raw
        # entries from offset[j], rounded up to 64 entries (256-byte aligned
        # starts); results are views into them
        offsets, total = [], 0
        for j in range(n):
            _check_fitness(ctx, spaces[j], fitness[j])
            offsets.append(total)
            total += (_n_raw(spaces[j]) + 63) // 64 * 64
        dev = torch.device("cuda", ctx.device)
        pr_all = torch.empty(max(total, 1), dtype=torch.float64, device=dev)
        min_all = torch.empty(max(total, 1), dtype=torch.int32, device=dev)
        pr_base, min_base = pr_all.data_ptr(), min_all.data_ptr()
        for j in range(n):
            sp, arr = _space(spaces[j])
            keep.append(arr)
            sp_arr[j] = sp
            fit_ptrs[j] = fitness[j].data_ptr()
            nb_arr[j] = _nb(nbs[j])
            prm_arr[j] = _params(ds[j], ps[j], tols[j], its[j], 0)
            pr_ptrs[j] = pr_base + 8 * offsets[j]
            min_ptrs[j] = min_base + 4 * offsets[j]
        rc = _abi.load().fl_analyze_batch(ctx.handle, n, sp_arr, fit_ptrs, nb_arr, prm_arr, pr_ptrs,
                                          min_ptrs, outs)
        _check(ctx, rc, "fl_analyze_batch", allow=(_abi.FL_ENOCONV, _abi.FL_EINVAL, _abi.FL_EOVERFLOW))
        results = []
        for j in range(n):
            info = outs[j].as_dict()
            N, M = int(info["n_valid"]), int(info["n_minima"])
            o = offsets[j]
            results.append(Result(pr_all[o:o + N], min_all[o:o + M], None, float(info["score"]), info))
        return results
    finally:
        if own:
            ctx.close()
