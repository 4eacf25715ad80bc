"""Benchmark: FFG + PageRank + C_p analyses on one MI355X.

One step is one whole analysis of the large synthetic space (10 parameters,
radices 12,10,6,5,4,4,3,3,3,3, 4 665 600 raw / 1 516 320 valid
configurations, Hamming neighbourhood, d = 0.85, p = 0.05): compaction, FFG
degree count, scan, CSR fill, PageRank power iteration to ||dr||_1 < 2e-7,
local minima and C_p, all in the HIP engine through the C ABI.  The fitness
vector is resident in HBM before the timed region.

value = FFG+PageRank edges traversed per second over the timed steps,
        sum(E * iterations) / wall time, in GTEPS.
roofline = the PageRank sweep kernel (which, in the engine's default lagged
        form, also does the step of the sweep before): the algorithmic bytes
        of one SpMV iteration, 20 N + 8 E, over its mean duration (and, as
        layout_model, the bytes its own layout moves: (28 + 8 W) N + 4 E for
        the slot sweep with W record words per node), from pairs of
        HIP events on the engine's stream around sweep launches of the timed
        steps (every 8th launch by default, so that the events barely slow
        the steps; launches after convergence, which exit at once, are not
        counted), against 8 TB/s HBM.  traffic = HBM bytes per launch from
        rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by the same counters
        on a plain copy (see --traffic-from), or null when the kernel source
        changed since they were taken.
cpu_baseline = the FP64 oracle on the same space at the same tolerance,
        single-threaded on the host.
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FFG+PageRank edges/s (GTEPS) & % HBM peak at 1M configs; p50/p99 per-space latency"
HBM_PEAK_GBS = 8000.0
# the server runs analyses of graphs above this many edges alone on its
# builder's stream, beside the batch (the 1.5 M-node space has 23 M)
SERVING_ALONE_EDGES = 1 << 22
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pr_iter_slots_large_traffic.json")
LOOP_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_batch_sweep_batched234_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2210_01465_amd", "csrc", "fl_kernels.hip")


def kernel_digest() -> str:
    with open(KERNEL_SRC, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def traffic_record(path: str, kernel: str):
    """A committed HBM traffic record (from rocprofv3 --pmc runs), or None when
    absent, taken on another kernel, or on a different kernel source."""
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_digest") != kernel_digest() or rec.get("kernel") != kernel:
        return None
    return rec


def measured_traffic(kernel: str):
    """HBM bytes per launch of the sweep kernel from the committed PMC runs."""
    rec = traffic_record(TRAFFIC_FILE, kernel)
    return rec.get("bytes_per_launch") if rec else None


def _pmc_per_launch(csv_dir: str, counter: str, kernel_part: str):
    """Mean counter value over the dispatches of kernels whose name contains
    kernel_part and whose value is at least a tenth of the largest (this
    drops the launches that exit at once after convergence)."""
    import csv
    import glob
    vals = []
    for f in glob.glob(os.path.join(csv_dir, "*counter_collection.csv")):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter and kernel_part in r["Kernel_Name"]:
                    vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no {counter} rows for {kernel_part} under {csv_dir}")
    top = max(vals)
    work = [v for v in vals if v >= 0.1 * top]
    return sum(work) / len(work), len(work)


def _pmc_total(csv_dir: str, counter: str, kernel_parts):
    """Sum of a counter over every dispatch of kernels whose name contains one
    of kernel_parts, and the number of those dispatches."""
    import csv
    import glob
    total, n = 0.0, 0
    for f in glob.glob(os.path.join(csv_dir, "*counter_collection.csv")):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter and any(k in r["Kernel_Name"] for k in kernel_parts):
                    total += float(r["Counter_Value"])
                    n += 1
    if n == 0:
        raise SystemExit(f"no {counter} rows for {kernel_parts} under {csv_dir}")
    return total, n


def trace_mean_us(trace_dir: str, kernel_part: str, floor_frac: float = 0.5):
    """Mean duration (us) of the working launches of a kernel in a rocprofv3
    --kernel-trace CSV: launches at least floor_frac of the longest (sweep
    launches after convergence exit at once, in about a fifth of a working
    launch's time)."""
    import csv
    import glob
    ds = []
    for f in glob.glob(os.path.join(trace_dir, "*kernel_trace.csv")):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if kernel_part in r["Kernel_Name"]:
                    ds.append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    if not ds:
        raise SystemExit(f"no kernel-trace rows for {kernel_part} under {trace_dir}")
    top = max(ds)
    work = [d for d in ds if d >= floor_frac * top]
    return sum(work) / len(work), len(work)


def _copy_factors(root: str, copy_bytes: int):
    cf, _ = _pmc_per_launch(os.path.join(root, "pmc_FETCH_SIZE_copy"), "FETCH_SIZE", "copyBuffer")
    cw, _ = _pmc_per_launch(os.path.join(root, "pmc_WRITE_SIZE_copy"), "WRITE_SIZE", "copyBuffer")
    return cf, cw, copy_bytes / (cf * 1024.0), copy_bytes / (cw * 1024.0)


def write_traffic(root: str, kernel_part: str, copy_bytes: int, command: str, trace_dir: str = "") -> dict:
    """HBM bytes per launch of the sweep kernel from four rocprofv3 --pmc runs
    under root: pmc_FETCH_SIZE and pmc_WRITE_SIZE (bench.py), and
    pmc_FETCH_SIZE_copy / pmc_WRITE_SIZE_copy (bench.py --copy-probe
    copy_bytes).  Each counter is scaled by copy_bytes over what it reads for
    the copy, which moves copy_bytes each way.  With trace_dir, the mean
    duration of the kernel's working launches in that --kernel-trace run is
    recorded too, so that the DRAM rate follows from the record alone."""
    fetch, n = _pmc_per_launch(os.path.join(root, "pmc_FETCH_SIZE"), "FETCH_SIZE", kernel_part)
    write, _ = _pmc_per_launch(os.path.join(root, "pmc_WRITE_SIZE"), "WRITE_SIZE", kernel_part)
    cf, cw, f_fac, w_fac = _copy_factors(root, copy_bytes)
    rec = {"kernel": kernel_part, "kernel_digest": kernel_digest(), "launches": n,
           "fetch_kib_per_launch": round(fetch, 1), "write_kib_per_launch": round(write, 1),
           "copy_bytes": copy_bytes, "copy_fetch_kib": round(cf, 1), "copy_write_kib": round(cw, 1),
           "fetch_factor": round(f_fac, 4), "write_factor": round(w_fac, 4),
           "bytes_per_launch": int(fetch * 1024 * f_fac + write * 1024 * w_fac),
           "command": command}
    if trace_dir:
        mean, nt = trace_mean_us(trace_dir, kernel_part)
        rec["kernel_trace_mean_us"] = round(mean, 3)
        rec["kernel_trace_launches"] = nt
        rec["dram_gb_per_s"] = round(rec["bytes_per_launch"] / (mean * 1e-6) / 1e9, 1)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    return rec


LOOP_KERNELS = ("k_batch_sweep<", "k_batch_finish<false>")


def write_loop_traffic(root: str, copy_bytes: int, runs: int, command: str) -> dict:
    """HBM bytes of one batched sweep loop (every k_batch_sweep and
    k_batch_finish<false> dispatch) from rocprofv3 --pmc runs of
    `bench.py --batched-loop-only` under root (pmc_loop_FETCH_SIZE,
    pmc_loop_WRITE_SIZE), which runs the loop `runs` times; scaled by the
    copy calibration as in write_traffic."""
    fetch, n = _pmc_total(os.path.join(root, "pmc_loop_FETCH_SIZE"), "FETCH_SIZE", LOOP_KERNELS)
    write, _ = _pmc_total(os.path.join(root, "pmc_loop_WRITE_SIZE"), "WRITE_SIZE", LOOP_KERNELS)
    cf, cw, f_fac, w_fac = _copy_factors(root, copy_bytes)
    rec = {"kernel": "+".join(LOOP_KERNELS), "kernel_digest": kernel_digest(), "dispatches": n, "runs": runs,
           "fetch_kib_per_loop": round(fetch / runs, 1), "write_kib_per_loop": round(write / runs, 1),
           "fetch_factor": round(f_fac, 4), "write_factor": round(w_fac, 4),
           "bytes_per_loop": int((fetch * 1024 * f_fac + write * 1024 * w_fac) / runs), "command": command}
    with open(LOOP_TRAFFIC_FILE, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    return rec


def workload(name: str):
    from paper_2210_01465_amd import synth
    return {"large": synth.large, "mid": synth.mid, "tiny": synth.tiny}[name]()


def host_cpu() -> str:
    """CPU model and logical CPU count of the host (for the baseline line)."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical CPUs visible"


def copy_bandwidth(n_bytes: int = 1 << 30, repeats: int = 10) -> dict:
    """Device-to-device copy of n_bytes, timed with HIP events: the HBM rate a
    plain streaming kernel reaches on this GPU (read + write bytes / time)."""
    import torch
    n = n_bytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(repeats):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / repeats
    gbs = 2 * n * 4 / s / 1e9
    del src, dst
    return {"bytes_per_copy": 2 * n * 4, "gb_per_s": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "how": f"torch device-to-device copy of {n * 4} bytes, {repeats} copies between HIP events"}


def _median(xs):
    xs = sorted(xs)
    return xs[len(xs) // 2] if len(xs) % 2 else 0.5 * (xs[len(xs) // 2 - 1] + xs[len(xs) // 2])


def oracle_timed(space, nb, damping, p, tol):
    """One whole oracle analysis, timed per phase: build (space, FFG, minima
    and the export of the graph to numpy), PageRank, C_p."""
    import oracle
    t0 = time.perf_counter()
    g = oracle.build_graph(space.radix, space.fitness_raw, {"hamming": 0, "adjacent": 1}[nb])
    t1 = time.perf_counter()
    r, it, _ = g.pagerank(damping, tol)
    t2 = time.perf_counter()
    score = g.score(r, p)[0]
    t3 = time.perf_counter()
    return g, r, it, score, {"build": t1 - t0, "pagerank": t2 - t1, "score": t3 - t2, "total": t3 - t0}


def cpu_baseline(space, nb, damping, p, tol, runs: int = 5):
    """The FP64 oracle on the same space at the same tolerance, single-threaded:
    the median of `runs` whole analyses, with the median of each phase."""
    times = [oracle_timed(space, nb, damping, p, tol) for _ in range(runs)]
    g, _, it = times[0][0], times[0][1], times[0][2]
    t = _median([x[4]["total"] for x in times])
    phases = {k: round(_median([x[4][k] for x in times]), 4) for k in ("build", "pagerank", "score")}
    return {"value": round(g.E * it / t / 1e9, 6), "unit": "GTEPS", "cores": 1, "kind": "oracle",
            "sample": f"{runs} whole analyses of the same space ({space.name}, N={g.N}, E={g.E}) at tol {tol:g}, "
                      f"{it} FP64 iterations each, single-threaded, on {host_cpu()}; value from the median "
                      f"({t:.2f} s)",
            "runs_s": [round(x[4]["total"], 4) for x in times], "median_s": round(t, 4), "phases_s": phases}


def analysis_bytes(n_raw, N, E, M, k):
    """Algorithmic bytes of one whole analysis: (8 n_raw + 36 N + 4 E) for the
    build, k (20 N + 8 E) for the power iteration, 12 M for C_p."""
    return (8 * n_raw + 36 * N + 4 * E) + k * (20 * N + 8 * E) + 12 * M


def configs_leg(ctx, damping, p, tol, repeats: int = 10):
    """The smaller workloads, each as one whole analysis on the GPU (median
    wall time of `repeats` analyses after 3 warm-ups, plan_create +
    execute, synchronised) against the FP64 oracle: the tiny space
    (Hamming) and the mid space under both neighbourhoods.  Per workload:
    sizes, iterations, GPU time, GTEPS, algorithmic % of HBM peak, CSR and
    minima bit-exactness, L1 and C_p error against the oracle at 1e-13, and
    the oracle's own single-threaded time at the GPU's tolerance (median of 3)."""
    import numpy as np
    import torch
    import oracle
    from paper_2210_01465_amd import api, synth
    out = {}
    for name, space, nb in (("tiny_hamming", synth.tiny(0), "hamming"), ("mid_hamming", synth.mid(), "hamming"),
                            ("mid_adjacent", synth.mid(), "adjacent")):
        fit = torch.from_numpy(space.fitness_raw).cuda()

        def run():
            plan = api.plan_create(ctx, space.radix, fit, nb)
            pr, mins, info = api.execute(plan, damping, p, tol=tol)
            return plan, pr, mins, info
        for _ in range(3):
            run()[0].close()
        ts = []
        for _ in range(repeats):
            t0 = time.perf_counter()
            plan, pr, mins, info = run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
            if _ < repeats - 1:
                plan.close()
        ex = {k: v.cpu().numpy() for k, v in api.plan_export(plan).items()}
        pr, mins = pr.cpu().numpy(), mins.cpu().numpy()
        plan.close()
        onb = {"hamming": 0, "adjacent": 1}[nb]
        ref = oracle.analyze(space.radix, space.fitness_raw, onb, damping, p, tol=1e-13)
        g = ref.graph
        t = _median(ts)
        N, E, M, k = int(info["n_valid"]), int(info["n_edges"]), int(info["n_minima"]), int(info["iterations"])
        o_ts = [oracle_timed(space, nb, damping, p, tol)[4]["total"] for _ in range(3)]
        out[name] = {"radix": list(space.radix), "n_raw": space.n_raw, "n_valid": N, "n_edges": E, "n_minima": M,
                     "iterations": k, "gpu_ms": round(t * 1e3, 4), "gteps": round(E * k / t / 1e9, 3),
                     "pct_hbm_alg": round(analysis_bytes(space.n_raw, N, E, M, k) / t / (HBM_PEAK_GBS * 1e9), 4),
                     "csr_exact": bool(np.array_equal(ex["row_ptr"], g.row_ptr)
                                       and np.array_equal(ex["col_idx"], g.col_idx)
                                       and np.array_equal(ex["valid_raw"], g.valid_raw)),
                     "minima_exact": bool(np.array_equal(mins, g.minima)),
                     "pagerank_l1": float(np.abs(pr - ref.pagerank).sum()),
                     "score_abs": abs(info["score"] - ref.score),
                     "oracle_1thread_ms": round(_median(o_ts) * 1e3, 3)}
    return out


def oracle_threads() -> int:
    """Host threads for oracle work spread over many spaces: the CPUs this
    process may run on, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def batched_oracle(spaces, results, damping, p, tol):
    """The FP64 oracle over the batched workload, spaces spread over host
    threads (the ctypes calls release the interpreter lock): wall time at the
    GPU's tolerance, and the worst error of the batched GPU results against
    the oracle at 1e-12."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import oracle
    threads = oracle_threads()

    def one(j, t):
        s = spaces[j]
        return oracle.analyze(s.radix, s.fitness_raw, oracle.HAMMING, damping, p, tol=t)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        timed = list(ex.map(lambda j: one(j, tol), range(len(spaces))))
    wall = time.perf_counter() - t0
    edges = sum(a.graph.E * a.iterations for a in timed)
    with ThreadPoolExecutor(threads) as ex:
        refs = list(ex.map(lambda j: one(j, 1e-12), range(len(spaces))))
    l1 = max(float(np.abs(r.pagerank.cpu().numpy() - a.pagerank).sum()) for r, a in zip(results, refs))
    cp = max(abs(r.score - a.score) for r, a in zip(results, refs))
    exact = all(np.array_equal(r.minima.cpu().numpy(), a.graph.minima) for r, a in zip(results, refs))
    return ({"ms": round(wall * 1e3, 3), "threads": threads, "gteps": round(edges / wall / 1e9, 4),
             "kind": "oracle", "sample": f"all {len(spaces)} spaces at tol {tol:g}, spread over {threads} host threads "
                                         f"on {host_cpu()}"},
            {"pagerank_l1_max": l1, "score_abs_max": cp, "minima_exact": exact})


def batched_autotune(spaces, fits, damping, p, tol, repeats: int = 3):
    """The autotuner on the batched workload, in a context of its own: fl_tune
    on every space (its shape class's per-bucket mapping and layout), then
    the 234 spaces through fl_analyze_batch with automatic layouts, against
    the same call in a fresh untuned context.  Reports the tuning time, the
    layouts chosen and both call times."""
    import collections
    import torch
    from paper_2210_01465_amd import api
    radices = [s.radix for s in spaces]

    def timed(ctx):
        api.analyze_batch(radices, fits, "hamming", damping, p, tol, ctx=ctx)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(repeats):
            res = api.analyze_batch(radices, fits, "hamming", damping, p, tol, ctx=ctx)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / repeats, res
    with api.Context(0) as fresh:
        t_plain, _ = timed(fresh)
    with api.Context(0) as ctx:
        chosen = collections.Counter()
        t0 = time.perf_counter()
        for s, f in zip(spaces, fits):
            plan = api.plan_create(ctx, s.radix, f, "hamming")
            chosen[{-1: "slots", -2: "binned"}.get(api.tune(plan, damping, sweeps=3)["best"], "csr")] += 1
            plan.close()
        tune_s = time.perf_counter() - t0
        t_tuned, res = timed(ctx)
        used = collections.Counter({-1: "slots", -2: "binned"}.get(r.info["row_mapping"], "csr") for r in res)
    return {"tune_ms": round(tune_s * 1e3, 1), "layout_chosen": dict(chosen), "layout_run": dict(used),
            "ms_untuned": round(t_plain * 1e3, 3), "ms_tuned": round(t_tuned * 1e3, 3),
            "all_ok": all(r.info["status"] == 0 for r in res)}


def batched_leg(ctx, damping, p, tol, repeats: int = 3):
    """234 spaces (26 shapes x 9 landscapes, N from 414 to 196k): one
    fl_analyze_batch over all of them against the same analyses run one at a
    time through fl_plan_create + fl_execute."""
    import torch
    from paper_2210_01465_amd import api, synth
    spaces = synth.batched()
    fits = [torch.from_numpy(s.fitness_raw).cuda() for s in spaces]
    radices = [s.radix for s in spaces]
    api.analyze_batch(radices, fits, "hamming", damping, p, tol, ctx=ctx)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(repeats):
        res = api.analyze_batch(radices, fits, "hamming", damping, p, tol, ctx=ctx)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / repeats
    edges = sum(r.info["n_edges"] * r.info["iterations"] for r in res)
    nodes = sum(r.info["n_valid"] for r in res)
    t0 = time.perf_counter()
    for s, f in zip(spaces, fits):
        plan = api.plan_create(ctx, s.radix, f, "hamming")
        api.execute(plan, damping, p, tol=tol)
        plan.close()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    oracle_cpu, accuracy = batched_oracle(spaces, res, damping, p, tol)
    tuned = batched_autotune(spaces, fits, damping, p, tol, repeats)
    return {"spaces": len(spaces), "n_valid_total": nodes, "ms_batched": round(t_batch * 1e3, 3),
            "ms_one_at_a_time": round(t_plain * 1e3, 3), "speedup": round(t_plain / t_batch, 3),
            "gteps_batched": round(edges / t_batch / 1e9, 3),
            "gteps_one_at_a_time": round(edges / t_plain / 1e9, 3),
            "all_ok": all(r.info["status"] == 0 for r in res),
            "accuracy": accuracy, "oracle_all_threads": oracle_cpu, "autotune": tuned,
            "sweep_loop": batched_sweep_rate(ctx, spaces, fits, damping, p, tol)}


def batched_sweep_rate(ctx, spaces, fits, damping, p, tol, sweeps_per_step: int = 16):
    """HBM rate of the batched sweep loop alone: every space's plan built
    first, all added to one batch (the small-member path off, so that every
    member's sweeps run inside the timed loop), stepped to the end.
    Algorithmic bytes are the slot sweep's per-sweep bytes ((20 + 8 W) N +
    4 E) times each member's iteration count; time is the batch's HIP-event
    device time around its sweep loops (batched sweeps and the per-member
    step kernel together).  The second of two identical runs is reported
    (the first captures the loop's graphs)."""
    import torch
    from paper_2210_01465_amd import api
    plans = [api.plan_create(ctx, s.radix, f, "hamming") for s, f in zip(spaces, fits)]
    try:
        for _ in range(2):
            batch = api.Batch(ctx)
            batch.set_small(0)
            for j, pl in enumerate(plans):
                batch.add(pl, damping, p, tol=tol, tag=j)
            infos = {}
            while True:
                running = batch.step(sweeps_per_step)
                for tag, _, _, info in batch.collect():
                    infos[tag] = info
                if running == 0 and len(infos) == len(plans):
                    break
            tm = batch.timing()
            batch.close()
        torch.cuda.synchronize()
        alg = spmv = 0
        for j, pl in enumerate(plans):
            sz = pl.sizes
            it, n, e = infos[j]["iterations"], int(sz["n_valid"]), int(sz["n_edges"])
            alg += it * ((20 + 8 * int(sz["mask_words"])) * n + 4 * e)
            spmv += it * (20 * n + 8 * e)
        gbs = alg / (tm["sweep_ms"] * 1e-3) / 1e9
        spmv_gbs = spmv / (tm["sweep_ms"] * 1e-3) / 1e9
        out = {"members": len(plans), "sweeps": tm["sweeps"], "device_ms": round(tm["sweep_ms"], 3),
               "alg_bytes": int(alg), "alg_formula": "sum over members of iterations x ((20 + 8 W) N + 4 E)",
               "gb_per_s": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
               "spmv_bytes": int(spmv), "spmv_formula": "sum over members of iterations x (20 N + 8 E)",
               "spmv_gb_per_s": round(spmv_gbs, 1), "spmv_frac_of_peak": round(spmv_gbs / HBM_PEAK_GBS, 4),
               "graph_launches": tm["graph_launches"], "graph_captures": tm["graph_captures"], "traffic": None}
        rec = traffic_record(LOOP_TRAFFIC_FILE, "+".join(LOOP_KERNELS))
        if rec:        # DRAM bytes of the same loop, from rocprofv3 counters
            dram = rec["bytes_per_loop"] / (tm["sweep_ms"] * 1e-3) / 1e9
            out.update(traffic=rec["bytes_per_loop"], dram_gb_per_s=round(dram, 1),
                       dram_frac_of_peak=round(dram / HBM_PEAK_GBS, 4))
        return out
    finally:
        for pl in plans:
            pl.close()


def _wall_ms(fn, repeats: int = 5):
    """Median wall time (ms) of fn() over repeats calls after one warm-up call;
    every call ends with the device idle (the calls synchronise)."""
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(repeats):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2] * 1e3


def landscape_leg(ctx, space, fit, nb: str, p: float):
    """The landscape figures on the large workload, wall time per call:
    the exact method at d = 1 and 0.85 (Jacobi sweeps to a fixed point), the C_p curve
    over p = 0..15 %, the naive metric with a 20-bin histogram; and one
    paper-shaped space analysed with its failures kept as nodes of fitness
    1e10 (build plus PageRank): the GEMM-shaped space with 78 % failed."""
    import numpy as np
    import torch
    from paper_2210_01465_amd import api, synth
    plan = api.plan_create(ctx, space.radix, fit, nb)
    try:
        res, exact_pr = {}, None
        for d, key in ((1.0, "exact_d1"), (0.85, "exact_d085")):
            pr, _, info = api.execute(plan, d, p, exact=True)
            exact_pr = pr
            ms = _wall_ms(lambda: api.execute(plan, d, p, exact=True, pagerank=pr))
            E = int(info["n_edges"])
            res[key] = {"ms": round(ms, 3), "sweeps": int(info["iterations"]), "score": info["score"],
                        "gteps": round(E * info["iterations"] / ms / 1e6, 3)}
        pr, _, info = api.execute(plan, 0.85, p)
        grid = [j / 100 for j in range(16)]
        res["score_curve_16"] = {"ms": round(_wall_ms(lambda: api.score_curve(plan, pr, grid)), 4),
                                 "n_minima": int(info["n_minima"])}
        res["naive_metric_20"] = {"ms": round(_wall_ms(lambda: api.naive_metric(plan, 20)), 4)}
    finally:
        plan.close()
    s = synth.batched()[18]                      # a GEMM-shaped space, 78 % of it failed
    f = np.array(s.fitness_raw, dtype=np.float32, copy=True)
    failed = float(np.isnan(f).mean())
    f[np.isnan(f)] = np.float32(1e10)
    f_dev = torch.from_numpy(f).cuda()
    out = {}

    def paper_mode():
        pl = api.plan_create(ctx, s.radix, f_dev, nb)
        _, _, inf = api.execute(pl, 0.85, p)
        pl.close()
        out.update(inf)
    ms = _wall_ms(paper_mode)
    res["paper_failure_mode"] = {"space": s.name, "radix": list(s.radix), "failed_frac": round(failed, 4),
                                 "ms": round(ms, 3), "n_valid": int(out["n_valid"]),
                                 "n_edges": int(out["n_edges"]), "n_minima": int(out["n_minima"]),
                                 "n_plateau": int(out["n_plateau"]), "iterations": int(out["iterations"])}
    return res, exact_pr.cpu().numpy()


def serving_stream(spaces, fits, large_space, large_fit, rate: float, seconds: float, seed: int = 5,
                   at_once: int = 0):
    """Requests of the serving mix: 98 % drawn uniformly from the batched
    spaces, 2 % the large space, damping uniform on {0.8, 0.85, 0.9},
    p = 0.05; Poisson arrivals at `rate` per second over `seconds` (seeded),
    or `at_once` requests all arriving at time 0."""
    import numpy as np
    from paper_2210_01465_amd import serve
    rng = np.random.default_rng(seed)
    times = [0.0] * at_once if at_once else serve.poisson_arrivals(rate, seconds, seed=seed)
    reqs = []
    for rid, t in enumerate(times):
        d = float(rng.choice([0.8, 0.85, 0.9]))
        if rng.random() < 0.02:
            reqs.append(serve.Request(t, rid, ("large", "hamming"), large_space.radix, large_fit,
                                      "hamming", d, 0.05))
        else:
            j = int(rng.integers(len(spaces)))
            reqs.append(serve.Request(t, rid, (j, "hamming"), spaces[j].radix, fits[j], "hamming", d, 0.05))
    return reqs


def serve_both(ctx, reqs, warm: float, cache: bool = True, alone_edges: int | None = SERVING_ALONE_EDGES,
               alone_when_idle: bool = True, plain: bool = True, sweeps_per_step: int = 16,
               alone_on_builder: bool = True):
    """One request stream through the continuous-batching server (FFG builds
    of cache misses, and analyses of graphs above alone_edges edges, on the
    builder thread's stream; requests that find it idle run alone at once,
    and with alone_on_builder a request the builder can take at once runs
    alone there instead of joining the batch)
    and through the one-at-a-time path, both with the same content-keyed
    plan cache (or both without one).  Returns (served summary, plain
    summary or None, server stats, served Done records)."""
    import torch
    from paper_2210_01465_amd import serve
    free, _ = torch.cuda.mem_get_info()
    budget = int(free * 0.5)
    backend = serve.GpuBackend(ctx, sweeps_per_step=sweeps_per_step, async_builds=True)
    srv = serve.Server(backend, hbm_budget=budget, cache_budget=None if cache else 0,
                       alone_when_idle=alone_when_idle, alone_edges=alone_edges,
                       alone_on_builder=alone_on_builder, switch_interval=1e-4)
    done = srv.run(reqs)
    torch.cuda.synchronize()
    served = serve.latency_summary(done, since=warm)
    paths = collections.Counter(d.path for d in done)
    stats = {"ffg_builds": int(srv.stats["built"]), "cache_hits": int(srv.stats["cache_hits"]),
             "build_waits": int(srv.stats["build_waits"]), "peak_bytes": int(srv.peak_bytes),
             "paths": {k: int(paths[k]) for k in ("batch", "alone", "builder")}}
    srv.close()
    backend.close()
    if not plain:
        return served, None, stats, done
    pb = serve.GpuBackend(ctx)
    plain = serve.latency_summary(serve.serve_plain(pb, reqs, cache_budget=budget // 2 if cache else 0),
                                  since=warm)
    pb.close()
    return served, plain, stats, done


def served_accuracy(done, spaces, large_space, limit: int = 300):
    """The first `limit` served results against the FP64 oracle at 1e-12
    (each distinct space and damping once, over host threads): worst L1 of
    the ranks, worst |C_p| error, minima exact."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import oracle
    sample = sorted(done, key=lambda d: d.rid)[:limit]
    # large requests too, wherever they fall in the stream
    sample += [d for d in done if d.rid not in {x.rid for x in sample} and d.info["n_valid"] > 10 ** 6][:2]
    keyed = {}
    for d in sample:
        key = ("large" if d.info["n_valid"] > 10 ** 6 else d.space_index, d.damping)
        keyed.setdefault(key, []).append(d)

    def ref(key):
        j, dmp = key
        s = large_space if j == "large" else spaces[j]
        return oracle.analyze(s.radix, s.fitness_raw, oracle.HAMMING, dmp, 0.05, tol=1e-12)
    with ThreadPoolExecutor(oracle_threads()) as ex:
        refs = dict(zip(keyed, ex.map(ref, list(keyed))))
    l1 = cp = 0.0
    exact = True
    for key, ds in keyed.items():
        a = refs[key]
        for d in ds:
            l1 = max(l1, float(np.abs(d.pagerank.cpu().numpy() - a.pagerank).sum()))
            cp = max(cp, abs(d.score - a.score))
            exact = exact and bool(np.array_equal(d.minima.cpu().numpy(), a.graph.minima))
    return {"requests": len(sample), "distinct": len(keyed), "pagerank_l1_max": l1, "score_abs_max": cp,
            "minima_exact": exact}


def serving_leg(ctx, large_space, large_fit, seconds: float, rates=(2000.0, 4000.0, 8000.0),
                sweep_seconds: float = 4.0, warm: float = 2.0):
    """The serving figures.  main: Poisson 1000 requests/s, `warm` s of
    warm-up then `seconds` measured, served against one at a time, both with
    the same plan cache.  rates: the same mix at higher rates (1 s warm-up,
    `sweep_seconds` measured); a rate is sustained when the measured
    throughput is at least 97 % of it.  saturation: 3000 requests all
    arriving at once (throughput at saturation).  cache_misses: 1000/s with
    no plan cache on either path, so every request builds its FFG (on the
    builder's stream for the server)."""
    import torch
    from paper_2210_01465_amd import synth
    spaces = synth.batched()
    fits = [torch.from_numpy(s.fitness_raw).cuda() for s in spaces]
    reqs = serving_stream(spaces, fits, large_space, large_fit, 1000.0, warm + seconds)
    served, plain, stats, done = serve_both(ctx, reqs, warm)
    by_rid = {r.rid: r for r in reqs}
    for d in done:
        r = by_rid[d.rid]
        d.space_index, d.damping = r.key[0], r.damping
    out = {"rate_per_s": 1000.0, "seconds": seconds, "warmup_s": warm, "requests": len(reqs),
           "served": served, "one_at_a_time": plain, **stats,
           "accuracy": served_accuracy(done, spaces, large_space)}
    del done
    sweep = {}
    best = {"served": 1000.0 if served["measured_throughput_per_s"] >= 970.0 else None,
            "one_at_a_time": 1000.0 if plain["measured_throughput_per_s"] >= 970.0 else None}
    for rate in rates:
        print(f"[bench] serving at {rate:g} requests/s", file=sys.stderr, flush=True)
        rq = serving_stream(spaces, fits, large_space, large_fit, rate, 1.0 + sweep_seconds, seed=6)
        sv, pl, st, _ = serve_both(ctx, rq, 1.0)
        sweep[str(int(rate))] = {"served": sv, "one_at_a_time": pl, **st}
        for name, summ in (("served", sv), ("one_at_a_time", pl)):
            if summ["measured_throughput_per_s"] >= 0.97 * rate:
                best[name] = max(best[name] or 0.0, rate)
    out["rates"] = sweep
    out["max_sustained_rate_per_s"] = best
    print("[bench] serving at saturation", file=sys.stderr, flush=True)
    rq = serving_stream(spaces, fits, large_space, large_fit, 0.0, 0.0, seed=7, at_once=3000)
    sv, pl, st, _ = serve_both(ctx, rq, 0.0)
    out["saturation"] = {"requests": len(rq), "served_per_s": sv["throughput_per_s"],
                         "one_at_a_time_per_s": pl["throughput_per_s"], "served_gteps": sv["gteps"],
                         "one_at_a_time_gteps": pl["gteps"], **st}
    print("[bench] serving without a plan cache", file=sys.stderr, flush=True)
    rq = serving_stream(spaces, fits, large_space, large_fit, 1000.0, 1.0 + sweep_seconds, seed=8)
    sv, pl, st, _ = serve_both(ctx, rq, 1.0, cache=False)
    out["cache_misses"] = {"rate_per_s": 1000.0, "served": sv, "one_at_a_time": pl, **st}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["large", "mid", "tiny"])
    ap.add_argument("--neighbourhood", default="hamming", choices=["hamming", "adjacent"])
    ap.add_argument("--row-mapping", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched leg (234 spaces in one fl_analyze_batch vs one at a time)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-configs", action="store_true", help="skip the tiny and mid workloads")
    ap.add_argument("--no-landscape", action="store_true",
                    help="skip the landscape figures (exact method, C_p curve, naive metric, failure mode)")
    ap.add_argument("--serving-seconds", type=float, default=10.0,
                    help="measured length of the Poisson request stream (after 2 s of warm-up)")
    ap.add_argument("--serving-warmup", type=float, default=2.0)
    ap.add_argument("--serving-rates", default="2000,4000,8000",
                    help="comma-separated request rates of the serving sweep (empty: none)")
    ap.add_argument("--serving-sweep-seconds", type=float, default=4.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes five times "
                         "(calibrates the HBM byte counters of a profiler)")
    ap.add_argument("--traffic-from", metavar="DIR",
                    help="write the sweep kernel's HBM traffic record from the rocprofv3 --pmc "
                         "runs under DIR (no GPU needed) and exit")
    ap.add_argument("--traffic-kernel", default="k_pr_iter_slots<2, true, true>")
    ap.add_argument("--trace-from", metavar="DIR", default="",
                    help="with --traffic-from: a rocprofv3 --kernel-trace run whose mean working-launch "
                         "duration of the kernel goes into the traffic record")
    ap.add_argument("--traffic-loop-from", metavar="DIR",
                    help="write the batched sweep loop's HBM traffic record from the rocprofv3 --pmc runs "
                         "of --batched-loop-only under DIR (no GPU needed) and exit")
    ap.add_argument("--batched-loop-only", action="store_true",
                    help="only run the batched sweep loop (234 prebuilt plans stepped to the end, twice); "
                         "for the profiler's byte counters")
    ap.add_argument("--traffic-copy-bytes", type=int, default=1 << 30)
    ap.add_argument("--traffic-command", default="")
    ap.add_argument("--sweep-event-every", type=int, default=0, metavar="N",
                    help="bracket every N-th sweep launch of the timed steps with its own HIP events and "
                         "take the roofline's launch time from those (0, the default: from the events "
                         "around each chunk of back-to-back sweep launches)")
    args = ap.parse_args()

    if args.traffic_from:
        print(json.dumps(write_traffic(args.traffic_from, args.traffic_kernel,
                                       args.traffic_copy_bytes, args.traffic_command, args.trace_from)))
        return
    if args.traffic_loop_from:
        print(json.dumps(write_loop_traffic(args.traffic_loop_from, args.traffic_copy_bytes, 2,
                                            args.traffic_command)))
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this engine has no multi-GPU path "
              "(independent spaces would be routed to GPUs whole; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2210_01465_amd import api

    if args.copy_probe:
        n = args.copy_probe // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 4, "copies": 5}), flush=True)
        return

    damping, p, tol = 0.85, 0.05, 2e-7
    if args.batched_loop_only:
        from paper_2210_01465_amd import synth
        ctx = api.Context(0)
        spaces = synth.batched()
        fits = [torch.from_numpy(s.fitness_raw).cuda() for s in spaces]
        print(json.dumps({"batched_sweep_loop": batched_sweep_rate(ctx, spaces, fits, damping, p, tol)}), flush=True)
        ctx.close()
        return
    space = workload(args.workload)
    print(f"[bench] workload {space.name} radix={space.radix}", file=sys.stderr, flush=True)
    fit = torch.from_numpy(space.fitness_raw).cuda()
    ctx = api.Context(0)
    n_raw = space.n_raw
    pr_buf = torch.empty(n_raw, dtype=torch.float64, device="cuda")
    min_buf = torch.empty(n_raw, dtype=torch.int32, device="cuda")

    tuning = None
    if args.row_mapping == 0:
        # autotune the sweep layout for this shape class (outside the timed
        # region, once per context, as a server would on a new shape class)
        plan = api.plan_create(ctx, space.radix, fit, args.neighbourhood)
        t0 = time.perf_counter()
        tuning = api.tune(plan, damping, sweeps=5)
        tuning["tune_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
        tuning["us_per_sweep"] = {str(k): round(v, 3) for k, v in tuning["us_per_sweep"].items()}
        plan.close()
        print(f"[bench] autotune: {tuning}", file=sys.stderr, flush=True)

    def step():
        plan = api.plan_create(ctx, space.radix, fit, args.neighbourhood)
        pr, mins, info = api.execute(plan, damping, p, tol=tol, row_mapping=args.row_mapping,
                                     pagerank=pr_buf, minima=min_buf)
        t = api.plan_timing(plan)
        plan.close()
        return info, t

    for _ in range(args.warmup):
        step()
    if args.sweep_event_every > 0:
        api.profile(ctx, args.sweep_event_every)
    torch.cuda.synchronize()
    infos, timings = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info, t = step()
        infos.append(info)
        timings.append(t)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    api.profile(ctx, 0)
    print(f"[bench] {args.steps} steps in {wall:.3f} s", file=sys.stderr, flush=True)

    info = infos[-1]
    N, E, M = info["n_valid"], info["n_edges"], info["n_minima"]
    edges = sum(i["n_edges"] * i["iterations"] for i in infos)
    gteps = edges / wall / 1e9
    if args.sweep_event_every > 0:  # sweep kernels that did work, each between its own events
        avg_launch_s = sum(t["sweep_ms"] for t in timings) / 1e3 / sum(t["sweeps_timed"] for t in timings)
    else:
        # events around each chunk of back-to-back sweep launches (the lagged
        # step launches no other kernel between them), over the sweeps that
        # did work: iterations + 2 per analysis (the step, and with it the
        # stop test, runs one sweep late, and one more sweep sees the stop)
        avg_launch_s = (sum(t["iterate_ms"] for t in timings) / 1e3
                        / sum(i["iterations"] + 2 for i in infos))
    # the PageRank SpMV's algorithmic bytes per iteration: y in, y out, x out,
    # out_deg, row_ptr (4 N each) and col_idx plus the x gathers (4 E each)
    bytes_per_launch = 20 * N + 8 * E
    if info["row_mapping"] == -1:   # slot sweep: records, y in/out, x out; x gathers (no col_idx)
        # lagged step: the previous iterate and g are read as well (8 N)
        layout_bytes = (28 + 8 * info["mask_words"]) * N + 4 * E
        layout_formula = f"(28 + 8 W) N + 4 E, W = {info['mask_words']} record words"
        buf = 16 * ((n_raw + 3) // 4) < 2 ** 31
        kernel = f"k_pr_iter_slots<{info['mask_words']}, {'true' if buf else 'false'}, true>"
    else:                           # CSR sweep reads the SpMV bytes, and 8 N more for the lagged step
        layout_bytes = bytes_per_launch + 8 * N
        layout_formula = "28 N + 8 E"
        kernel = ("k_pr_iter_binned<true>" if info["row_mapping"] == -2
                  else f"k_pr_iter_csr<{info['row_mapping']}, true>")
    achieved = bytes_per_launch / avg_launch_s / 1e9
    traffic_rec = traffic_record(TRAFFIC_FILE, kernel)
    traffic = traffic_rec.get("bytes_per_launch") if traffic_rec else None
    alg_bytes = analysis_bytes(n_raw, N, E, M, info["iterations"])
    step_s = wall / args.steps

    out = {
        "metric": METRIC,
        "value": round(gteps, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{space.name}: radices {','.join(map(str, space.radix))}, "
                               f"{n_raw} raw / {N} valid configs, {args.neighbourhood}, "
                               f"d={damping}, p={p}, tol={tol:g}",
                   "n_raw": n_raw, "n_valid": N, "n_edges": E, "n_minima": M,
                   "iterations": info["iterations"], "row_mapping": info["row_mapping"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "kernel": kernel,
                     "bytes_per_launch": bytes_per_launch,
                     "bytes_formula": "20 N + 8 E (algorithmic bytes of one PageRank SpMV iteration); "
                                      "frac = bytes_per_launch / avg_launch_us / peak",
                     "avg_launch_us": round(avg_launch_s * 1e6, 3),
                     "layout_model": {"formula": layout_formula, "bytes_per_launch": layout_bytes,
                                      "achieved": round(layout_bytes / avg_launch_s / 1e9, 1),
                                      "frac": round(layout_bytes / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4)},
                     "dram": None if not traffic_rec else {
                         "bytes_per_launch": traffic,
                         "achieved_live": round(traffic / avg_launch_s / 1e9, 1),
                         "frac_live": round(traffic / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4),
                         "kernel_trace_mean_us": traffic_rec.get("kernel_trace_mean_us"),
                         "achieved_trace": traffic_rec.get("dram_gb_per_s"),
                         "frac_trace": (round(traffic_rec["dram_gb_per_s"] / HBM_PEAK_GBS, 4)
                                        if traffic_rec.get("dram_gb_per_s") else None)},
                     "timing": ("HIP events on the engine's stream around each chunk of back-to-back sweep "
                                "launches of the timed steps, over the sweeps that did work "
                                f"({sum(i['iterations'] + 2 for i in infos)})")
                               if args.sweep_event_every <= 0
                               else f"HIP events around every {args.sweep_event_every}th sweep launch "
                                    f"of the timed steps ({sum(t['sweeps_timed'] for t in timings)} "
                                    f"working launches)"},
        "phases_ms": {k: round(float(np.mean([t[k] for t in timings])), 4)
                      for k in ("build_ms", "pagerank_ms", "iterate_ms", "sweep_ms", "score_ms")},
        "analysis_pct_hbm_alg": round(alg_bytes / step_s / (HBM_PEAK_GBS * 1e9), 4),
        # edges x iterations over the PageRank phase alone (build and score excluded)
        "gteps_spmv": round(E * info["iterations"] / (float(np.mean([t["pagerank_ms"] for t in timings])) / 1e3)
                            / 1e9, 3),
        "score": info["score"],
    }
    out["hbm_copy"] = copy_bandwidth()
    if tuning is not None:
        out["autotune"] = tuning

    if not args.no_configs:
        print("[bench] tiny and mid workloads", file=sys.stderr, flush=True)
        out["configs"] = configs_leg(ctx, damping, p, tol)

    if not args.no_batched:
        print("[bench] batched leg", file=sys.stderr, flush=True)
        out["batched"] = batched_leg(ctx, damping, p, tol)

    exact_pr = None
    if not args.no_landscape:
        print("[bench] landscape figures", file=sys.stderr, flush=True)
        out["landscape"], exact_pr = landscape_leg(ctx, space, fit, args.neighbourhood, p)

    if not args.no_serving:
        print("[bench] serving leg", file=sys.stderr, flush=True)
        rates = tuple(float(x) for x in args.serving_rates.split(",") if x.strip())
        out["serving"] = serving_leg(ctx, space, fit, args.serving_seconds, rates=rates,
                                     sweep_seconds=args.serving_sweep_seconds, warm=args.serving_warmup)

    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle, median of 5)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(space, args.neighbourhood, damping, p, tol)
    if not args.no_accuracy:
        print("[bench] accuracy vs FP64 oracle at 1e-13", file=sys.stderr, flush=True)
        import oracle
        ref = oracle.analyze(space.radix, space.fitness_raw, {"hamming": 0, "adjacent": 1}[args.neighbourhood],
                             damping, p, tol=1e-13)
        pr = pr_buf[:N].cpu().numpy()
        out["accuracy"] = {"pagerank_l1": float(np.abs(pr - ref.pagerank).sum()),
                           "score_abs": abs(info["score"] - ref.score),
                           "minima_exact": bool(np.array_equal(min_buf[:M].cpu().numpy(),
                                                               ref.graph.minima))}
        if exact_pr is not None:      # the exact method at d = 0.85 against the same reference
            out["accuracy"]["exact_pagerank_l1"] = float(np.abs(exact_pr - ref.pagerank).sum())
            out["accuracy"]["exact_score_abs"] = abs(out["landscape"]["exact_d085"]["score"] - ref.score)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
