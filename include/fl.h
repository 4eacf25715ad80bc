/*
 * fl.h - C ABI of the MI355X fitness-flow-graph landscape engine.
 *
 * The engine computes, for one discrete search space with a runtime per
 * configuration, the landscape metric of Schoonhoven, van Werkhoven and
 * Batenburg, "Benchmarking optimization algorithms for auto-tuning GPU
 * kernels":
 *   - the search space X = S_1 x ... x S_n and its valid points   (Sec. III-B)
 *   - the Hamming (eq. 2) or adjacent neighbourhood                 (Sec. III-B)
 *   - the fitness flow graph (FFG): an edge from every point to each
 *     neighbour with strictly lower fitness                          (Sec. VII-B)
 *   - PageRank centrality of the FFG by power iteration             (Sec. VII-B)
 *   - the local minima (FFG sinks)                                   (Sec. III-B)
 *   - the p-proportion of centrality C_p                            (Sec. VII-B, eq. 3)
 *
 * Conventions shared by every call:
 *   - Every call returns fl_status.  No C++ exception crosses the ABI.  On an
 *     error the context keeps a message, readable with fl_last_error().
 *   - Pointers named d_* are device pointers (HIP device memory of the
 *     context's device); every other pointer is a host pointer.
 *   - All device work is ordered on the context's stream.  Input buffers are
 *     borrowed for the duration of the call; output buffers are owned by the
 *     caller.  Calls that return sizes or scores synchronise that stream.
 *   - A context is not thread-safe: serialise calls that share one.
 *   - Configurations are numbered in mixed radix with parameter 0 the most
 *     significant digit: raw index I(x) = sum_i x_i * prod_{j>i} radix_j,
 *     x_i the position of the value in the list S_i.  Valid points get node
 *     ids 0..N-1 in ascending raw index.
 *   - A configuration is a valid point iff its fitness is finite and > 0; the
 *     caller marks configurations that violate a constraint or failed with
 *     NaN or +inf.  A fitness <= 0 or -inf is an error (FL_EINVAL).
 *   - Two fitness values are compared exactly in float32; equal neighbours
 *     get no edge.  A local minimum is a node with no strictly better
 *     neighbour, i.e. an FFG sink (isolated valid points included).
 *   - PageRank is the stationary vector (sum 1) of
 *       G = d (P + (1/N) 1 s^T) + ((1-d)/N) 1 1^T,
 *     P[w,u] = 1/out_deg(u) per edge u->w, s the sink indicator: damping d,
 *     uniform teleport, and the mass of a sink spread uniformly.
 */
#ifndef FL_H
#define FL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FL_OK = 0,
    FL_EINVAL = -1,     /* invalid argument or fitness value */
    FL_ENOMEM = -2,     /* device or host allocation failed */
    FL_EHIP = -3,       /* a HIP runtime call failed */
    FL_ENOCONV = -4,    /* max_iter reached before the tolerance; outputs still written */
    FL_EOVERFLOW = -5,  /* n_raw or the edge count is >= 2^31 */
    FL_EBUSY = -6,      /* reserved for admission control */
    FL_ENOTIMPL = -7    /* entry point not available in this build */
} fl_status;

typedef enum {
    FL_NB_HAMMING = 0,  /* differ in exactly one parameter (Sec. III-B, eq. 2) */
    FL_NB_ADJACENT = 1  /* ... and that parameter's value is next in its list (Sec. III-B) */
} fl_neighbourhood;

/* A search space X = S_1 x ... x S_n (Sec. III-B).  radix[i] = |S_i| >= 1,
 * 1 <= n_params <= 32, prod radix < 2^31.  Host pointer, borrowed. */
typedef struct {
    int32_t n_params;
    const int32_t *radix;
} fl_space;

/* Analysis parameters.
 *   damping   d in (0,1); the paper leaves d open, 0.85 is the usual value.
 *   p         proportion for C_p as a fraction (0.05 = 5 %), p >= 0 and finite.
 *   tol_l1    stop when ||r_{k+1} - r_k||_1 < tol_l1 (0 => 2e-7).
 *   max_iter  iteration cap (0 => 1000); reaching it gives FL_ENOCONV.
 *   row_mapping  layout of the PageRank sweep: 0 = automatic (the layout
 *             fl_tune cached for the plan's shape class, else FL_ROWS_SLOTS
 *             where available, else FL_ROWS_BINNED);
 *             FL_ROWS_SLOTS = one node per lane over the in-edge slot
 *             records (needs at most 256 candidate slots per node);
 *             FL_ROWS_BINNED = the CSR with rows binned by in-degree into
 *             8 buckets (0; [2^(b-1), 2^b) for b = 1..6; 64 and more), each
 *             bucket with its own lanes per row and rows per tile (the
 *             mapping fl_tune chose for the plan's shape class, else about a
 *             quarter of the bucket's largest in-degree in lanes);
 *             1, 2, 4, 8, 16, 32 or 64 = that many lanes per row over the
 *             CSR.  Every layout sums a row's terms in ascending source
 *             order (one lane per row: sequentially; several: lane partial
 *             sums reduced by a fixed tree): with FL_STEP_SEPARATE the
 *             slot layout and the one-lane CSR layout give the same ranks
 *             bit for bit (the lagged step sums per workgroup, and their
 *             number depends on the layout's kernel). */
#define FL_ROWS_SLOTS (-1)
#define FL_ROWS_BINNED (-2)
#define FL_TUNE_LAYOUTS 9
/* flags: 0, or FL_STEP_SEPARATE.  By default fl_execute and
 *             fl_execute_exact run the sweeps back to back and each sweep
 *             also does the step (sums, residual, stop test) of the one
 *             before; the power iteration then stores each iterate without
 *             its constant teleport-and-sink term and adds it one step
 *             later.  Same iterates in exact arithmetic, same iteration
 *             count up to rounding at the tolerance; one or two more sweeps
 *             run past the stop.  FL_STEP_SEPARATE runs a step kernel after
 *             every sweep instead, the order of sums that batch members
 *             (fl_batch_step, fl_analyze_batch) use: a plan run that way
 *             gives its batch results bit for bit.
 *   reserved  must be 0. */
#define FL_STEP_SEPARATE 1
typedef struct {
    double damping;
    double p;
    double tol_l1;
    int32_t max_iter;
    int32_t row_mapping;
    int32_t flags;
    int32_t reserved;
} fl_params;

/* Sizes and results of one analysis. */
typedef struct {
    int64_t n_raw;       /* prod radix */
    int64_t n_valid;     /* N, valid points = FFG nodes */
    int64_t n_edges;     /* E, FFG edges */
    int64_t n_minima;    /* M, local minima = sinks */
    int32_t iterations;  /* PageRank iterations run */
    int32_t row_mapping; /* sweep layout used (FL_ROWS_SLOTS or lanes per CSR row) */
    int32_t n_slots;     /* candidate neighbour slots per node (2 per neighbour offset) */
    int32_t mask_words;  /* 64-bit words of a node record (0: too many slots, CSR sweep only) */
    int32_t status;      /* fl_status of this analysis (batched calls) */
    int32_t n_plateau;   /* local minima with a neighbour of equal fitness */
    double residual_l1;  /* ||r_k - r_{k-1}||_1 of the last iteration */
    double f_opt;        /* minimum valid fitness */
    double score;        /* C_p */
    double mass_minima;  /* sum of PageRank over L(X) */
    double mass_near;    /* sum of PageRank over L_p(X) */
} fl_summary;

/* Device time of the phases of the last fl_execute / fl_plan_create on a
 * plan, from HIP events on the context's stream (milliseconds). */
typedef struct {
    double build_ms;     /* compaction, degree count, scan, CSR fill */
    double pagerank_ms;  /* initialisation + all power iterations, host round trips included */
    double iterate_ms;   /* device time of the iteration launches alone (sum over chunks) */
    double score_ms;     /* output of the ranks, minima and C_p */
    int32_t iterations;  /* iteration kernels that did work */
    int32_t launches;    /* iteration kernels launched (extra ones exit at once) */
    double sweep_ms;     /* device time of the timed sweep kernels that did
                            work (the edge gathers alone), summed; measured
                            only while fl_profile is on, else 0 */
    int32_t sweeps_timed; /* number of sweeps summed in sweep_ms */
    int32_t reserved;
} fl_timing;

typedef struct fl_ctx fl_ctx;
typedef struct fl_plan fl_plan;

/* Create a context on HIP device `device`, ordering all work on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  The stream stays owned by the
 * caller and must outlive the context. */
fl_status fl_create(fl_ctx **ctx, int device, void *hip_stream);

/* Release the context and every device buffer it caches.  Plans created on it
 * must be destroyed first. */
fl_status fl_destroy(fl_ctx *ctx);

/* Message of the last failed call on ctx (owned by ctx, valid until the next
 * call).  Never NULL. */
const char *fl_last_error(const fl_ctx *ctx);

/* Phase 1: build the FFG of a space (Sec. III-B, Sec. VII-B) - compaction of
 * the valid points, neighbour enumeration, in/out degrees, prefix scan and
 * CSR fill.  Independent of damping and p.
 *   d_fitness_raw  device float32[prod radix] in raw order; borrowed.
 *   out            receives a plan owned by the library (fl_plan_destroy).
 *   sizes          receives n_raw, n_valid, n_edges, n_minima, f_opt.
 * A space with more than 256 candidate slots (no slot records) also gets
 * its rows binned by in-degree here, for the binned sweep.
 * Errors: FL_EINVAL (space, neighbourhood, a fitness <= 0 or -inf, no valid
 * point), FL_EOVERFLOW, FL_ENOMEM, FL_EHIP.  Synchronises the stream. */
fl_status fl_plan_create(fl_ctx *ctx, const fl_space *space, const float *d_fitness_raw,
                         fl_neighbourhood nb, fl_plan **out, fl_summary *sizes);

/* Phase 2: PageRank centrality on the plan's FFG, the local minima and C_p
 * (Sec. VII-B, eq. 3).
 *   d_pagerank  device double[N]: centrality of every node, sums to 1.
 *   d_minima    device int32[M]: node ids of the local minima, ascending.
 *   out         receives the full summary.
 * Errors: FL_EINVAL (damping not in (0,1), p < 0 or not finite, tol_l1 < 0,
 * max_iter < 0, bad row_mapping or FL_ROWS_SLOTS on a space with more than
 * 256 candidate slots), FL_ENOCONV (outputs written, summary holds
 * the residual), FL_ENOMEM, FL_EHIP.  Synchronises the stream. */
fl_status fl_execute(fl_ctx *ctx, fl_plan *plan, const fl_params *params,
                     double *d_pagerank, int32_t *d_minima, fl_summary *out);

/* Exact PageRank without a tolerance (Sec. VII-B): every FFG edge lowers the
 * fitness, so P is nilpotent and the stationary vector is r = u / sum(u)
 * with u = 1 + d P u.  Jacobi sweeps u <- 1 + d P u (the same sweep kernels
 * as fl_execute) stop changing after at most (longest path + 1) sweeps
 * (sooner where the weight of a distant ancestor, d^k times the product
 * of 1/out_deg along the path, falls below FP32 resolution),
 * detected by a sweep that changes no value; r, the minima and C_p are then
 * written as by fl_execute.  damping may be 1: then u(m) / N for a minimum m is the
 * probability that a descent from a uniformly random start, moving to a
 * uniformly random better neighbour, ends in m, and C_p is the probability
 * that it ends within (1 + p) f_opt.  tol_l1 is ignored; max_iter 0 means
 * N + 2; summary.iterations = sweeps run (at most longest path + 2).  Errors as
 * fl_execute (FL_EINVAL for damping outside (0, 1]). */
fl_status fl_execute_exact(fl_ctx *ctx, fl_plan *plan, const fl_params *params, double *d_pagerank,
                           int32_t *d_minima, fl_summary *out);

/* Copy the plan's FFG out (any pointer may be NULL):
 *   d_valid_raw int32[N]   node id -> raw index
 *   d_row_ptr   int32[N+1] CSR over in-edges: sources of node w are
 *   d_col_idx   int32[E]     d_col_idx[d_row_ptr[w] .. d_row_ptr[w+1]), ascending
 *   d_out_deg   int32[N]   number of strictly better neighbours
 * Stream-ordered, does not synchronise. */
fl_status fl_plan_export(fl_ctx *ctx, const fl_plan *plan, int32_t *d_valid_raw,
                         int32_t *d_row_ptr, int32_t *d_col_idx, int32_t *d_out_deg);

/* Autotuner.  First, per in-degree bucket of the plan (see FL_ROWS_BINNED):
 * time `sweeps` binned sweeps over that bucket's rows alone for every lanes
 * per row L in 1, 2, ..., up to the bucket's largest in-degree (64 at most)
 * and every tile of T = 1 or 4 blocks of 256 / L rows, and keep the fastest
 * (L, T) of each bucket as the shape class's bucket mapping.  Then time every
 * sweep layout the plan allows (the slot sweep, the CSR sweep with 1, 2, 4,
 * 8, 16, 32, 64 lanes per row, the binned sweep with that mapping) for
 * `sweeps` forced power-iteration sweeps each (HIP events, after one warm-up
 * sweep), store the fastest in the context's tuning cache under the plan's
 * shape class (node-record width, neighbourhood, log2 N, mean in-degree) and
 * return it in *best.  us_per_sweep (may be NULL) receives FL_TUNE_LAYOUTS
 * times in microseconds in that layout order, -1 where a layout does not
 * apply.  Afterwards fl_execute and fl_batch_add with row_mapping 0 use the
 * cached layout (and FL_ROWS_BINNED the cached mapping) for plans of the
 * same shape class.  The plan's iterate buffers are overwritten; outputs of
 * earlier fl_execute calls are not touched.  Synchronises the stream. */
fl_status fl_tune(fl_ctx *ctx, fl_plan *plan, const fl_params *params, int32_t sweeps, int32_t *best,
                  double *us_per_sweep);

/* The in-degree bucket mapping the context holds for the plan's shape class
 * (tuned by fl_tune, else the default; see FL_ROWS_BINNED) and the plan's
 * rows per bucket.  lanes, blocks (int32[8]) and rows (int64[8]) are host
 * arrays, any may be NULL.  Synchronises the stream when rows is given. */
fl_status fl_bucket_map(fl_ctx *ctx, const fl_plan *plan, int32_t *lanes, int32_t *blocks, int64_t *rows);

/* C_p curve (Sec. VII-B, eq. 3; the paper plots C_p for p = 0, 1, ..., 15 %):
 * scores[j] = C_p for p = p_values[j] (fractions >= 0), from the ranks
 * d_pagerank (double[N], device) that fl_execute wrote for this plan.  One
 * launch for all proportions; the thresholds (1 + p) f_opt and the rank
 * sums are FP64, as in fl_execute.  p_values and scores are host arrays of
 * n_p entries, 1 <= n_p <= 4096.  Errors: FL_EINVAL (bad argument, p < 0 or
 * not finite), FL_EHIP.  Synchronises the stream. */
fl_status fl_score_curve(fl_ctx *ctx, const fl_plan *plan, const double *d_pagerank, int32_t n_p,
                         const double *p_values, double *scores);

/* Naive metric (Sec. VII-A): the fraction of optimal fitness f_opt / f(m) of
 * every local minimum m.  d_ratio (device double[M], may be NULL) receives
 * it in ascending node id of the minima; hist (host int64[n_bins], may be
 * NULL) the number of minima in each of n_bins equal bins of [0, 1], bin
 * min(floor(ratio * n_bins), n_bins - 1), computed in FP64.  1 <= n_bins <=
 * 65536.  Errors: FL_EINVAL, FL_ENOMEM, FL_EHIP.  Synchronises the stream. */
fl_status fl_naive_metric(fl_ctx *ctx, const fl_plan *plan, double *d_ratio, int32_t n_bins, int64_t *hist);

/* Sweep profiling: while `every` > 0, fl_execute brackets every every-th
 * sweep kernel launch of an analysis (the 0th, every-th, ...) with a pair of
 * HIP events on the context's stream and reports the summed device time of
 * those that did work in fl_timing.sweep_ms (count in sweeps_timed).  Each
 * timed sweep costs a few microseconds of device time for the events;
 * every = 0 (the default) turns it off.  FL_EINVAL for every < 0. */
fl_status fl_profile(fl_ctx *ctx, int32_t every);

/* Phase timings of the plan's last build and execute (see fl_timing). */
fl_status fl_plan_timing(fl_ctx *ctx, const fl_plan *plan, fl_timing *out);

/* Release a plan; its device buffers return to the context's cache. */
fl_status fl_plan_destroy(fl_ctx *ctx, fl_plan *plan);

/* One-shot analysis: fl_plan_create + fl_execute + fl_plan_export of the
 * node map + fl_plan_destroy.  Output buffers are sized by the upper bound
 * n_raw = prod radix: d_pagerank double[n_raw], d_minima int32[n_raw],
 * d_valid_raw int32[n_raw] (may be NULL); only the first N / M entries are
 * written.  Errors as fl_plan_create and fl_execute. */
fl_status fl_analyze(fl_ctx *ctx, const fl_space *space, const float *d_fitness_raw,
                     fl_neighbourhood nb, const fl_params *params, double *d_pagerank,
                     int32_t *d_minima, int32_t *d_valid_raw, fl_summary *out);

/* fl_analyze without any device allocation, for callers that cannot allocate
 * device memory (code that runs while a HIP graph is being captured, serving
 * loops with a fixed memory budget, harnesses that forbid hipMalloc).
 * Same arguments, outputs, results and errors as fl_analyze; the results
 * equal fl_analyze's bit for bit.  Every device buffer the analysis needs
 * (compaction, degrees, node records, CSR, iterates, partial sums, state)
 * is carved from one array of 64 MiB that the library holds on every device
 * it runs on until the process ends; the call makes no hipMalloc, hipFree
 * or event call and no host heap allocation on success.  Limit: about
 * 20 n_raw + (28 + 8 W) N + 4 E bytes plus small tables must fit in the
 * 64 MiB (W node-record words): spaces up to about a million raw
 * configurations with tens of millions of edges.  A space whose raw size
 * alone (20 n_raw bytes) exceeds it is rejected with FL_EINVAL before any
 * launch; one whose FFG turns out too large is rejected with FL_EINVAL
 * after the degree count (fl_last_error names the limit).  The array keeps
 * the last call's contents; everything that must start at zero is cleared
 * by the call.  All calls on one device share the array: calls that
 * overlap on one device (other contexts or streams, other threads) race
 * and must be serialised by the caller.  Synchronises the stream. */
fl_status fl_analyze_noalloc(fl_ctx *ctx, const fl_space *space, const float *d_fitness_raw,
                             fl_neighbourhood nb, const fl_params *params, double *d_pagerank,
                             int32_t *d_minima, int32_t *d_valid_raw, fl_summary *out);

/* ---- Batches: many spaces in one segmented PageRank (continuous batching) ----
 *
 * A batch runs the power iteration of many plans together: every sweep is one
 * segmented launch over the tiles of all running members (one launch per
 * node-record width of the slot-sweep members, one for the binned members),
 * followed by one launch that finishes the step of every member.  Each member keeps its own damping, tolerance, iteration count and
 * stop flag, and its results equal those of fl_execute with the slot sweep
 * (row_mapping FL_ROWS_SLOTS, flags FL_STEP_SEPARATE) bit for bit, whatever
 * else runs in the batch.  A batch ignores FL_STEP_SEPARATE in the
 * parameters: its members always take a step kernel per sweep.
 * Members join (fl_batch_add) and leave (fl_batch_collect) between steps.
 * A member reads its plan's FFG and keeps its own iterate vectors (taken
 * from the context's device cache at fl_batch_add, returned when it leaves),
 * so one plan may be a member several times at once (say with different
 * damping or p), in one or several batches; it must stay alive while it is
 * a member.  The plan may come from another context on the same device (for
 * example one that builds FFGs on a second stream): its build must be
 * complete (fl_plan_create has returned), and it is still destroyed through
 * its own context.  fl_execute on a plan does not disturb its batch members. */
typedef struct fl_batch fl_batch;

fl_status fl_batch_create(fl_ctx *ctx, fl_batch **out);

/* Release the batch (not its plans).  Synchronises the stream. */
fl_status fl_batch_destroy(fl_ctx *ctx, fl_batch *batch);

/* Add a plan as a member; it starts at the next fl_batch_step.  The outputs
 * (d_pagerank double[N], d_minima int32[M]) are caller-owned device buffers
 * written when the member finishes; `tag` is returned by fl_batch_collect.
 * The member holds 8 n_raw + 8 N + 24 ceil(N/256) + 80 bytes of device
 * memory of its own while it is in the batch.
 * A member runs the slot sweep (FL_ROWS_SLOTS) or the binned sweep
 * (FL_ROWS_BINNED); row_mapping 0 takes the binned sweep where fl_tune
 * chose it for the plan's shape class in this context or where the slot
 * sweep cannot take the space, else the slot sweep (a tuned lanes-per-row
 * CSR layout wins on a lone space by spreading it over more workgroups; in
 * a batch the other members supply that parallelism).  A binned member
 * sweeps the plan's binned rows (built here with the class's tuned mapping
 * when the plan belongs to this context; a plan of another context must
 * already have them, as plans without slot records do).  Its results equal
 * fl_execute with FL_ROWS_BINNED, FL_STEP_SEPARATE and the same mapping bit
 * for bit.
 * Errors: FL_EINVAL (bad parameters, a row_mapping other than 0,
 * FL_ROWS_SLOTS or FL_ROWS_BINNED, FL_ROWS_SLOTS for a space the slot sweep
 * cannot take), FL_ENOMEM, FL_EHIP. */
fl_status fl_batch_add(fl_ctx *ctx, fl_batch *batch, fl_plan *plan, const fl_params *params,
                       double *d_pagerank, int32_t *d_minima, int64_t tag);

/* Run up to `sweeps` power-iteration sweeps (Sec. VII-B) for every running
 * member (up to 4 x `sweeps` for small members, see fl_batch_set_small);
 * members that converge or reach max_iter finish: their ranks,
 * minima and C_p (Sec. VII-B, eq. 3) are written.  *n_running receives the
 * number of members not yet finished.  The sweep loop of a step (per sweep:
 * one launch per node-record width, then the step launch) is captured once
 * per launch shape (the number of sweeps and grid sizes rounded to powers of
 * two) in a HIP graph and replayed by later steps of that shape; the batch
 * keeps the graphs of its 256 most recently used shapes and drops them all
 * when its tables grow.  Member lists and their lengths live in device
 * memory, so members may join and leave between replays.  Synchronises the
 * stream. */
fl_status fl_batch_step(fl_ctx *ctx, fl_batch *batch, int32_t sweeps, int32_t *n_running);

/* Remove up to `max` finished members: their tags and summaries (status
 * FL_OK or FL_ENOCONV in out[j].status).  *n_out receives the count. */
fl_status fl_batch_collect(fl_ctx *ctx, fl_batch *batch, int32_t max, int64_t *tags, fl_summary *out,
                           int32_t *n_out);

/* Sweeps run and device time of the sweep launches (HIP events) so far;
 * graph_launches / graph_captures (may be NULL): steps that replayed the
 * captured sweep loop and captures made. */
fl_status fl_batch_timing(fl_ctx *ctx, const fl_batch *batch, int64_t *sweeps, double *sweep_ms,
                          int64_t *graph_launches, int64_t *graph_captures);

/* Use the captured HIP graph for the sweep loop (enable != 0, the default)
 * or launch its kernels one by one.  Results are identical either way. */
fl_status fl_batch_set_graphs(fl_ctx *ctx, fl_batch *batch, int32_t enable);

/* Members of at most max_tiles tiles of 256 nodes (default 16, i.e. up to
 * 4096 nodes; 0 = none; at most 64) iterate inside one workgroup each: one
 * launch per record width and step runs up to 4 x `sweeps` of their sweeps
 * and steps back to back (until they stop), on a second stream of the
 * batch, while the other members' sweep loop runs on the context's stream.
 * Their results equal the plain slot sweep's bit for bit as well.  Takes
 * effect at the next fl_batch_step. */
fl_status fl_batch_set_small(fl_ctx *ctx, fl_batch *batch, int32_t max_tiles);

/* One-shot batched analysis of n_spaces spaces (Sec. VII-B for each): the
 * FFGs are built together, each build stage one launch for all spaces (a
 * table of per-space descriptors; one host synchronisation per stage), then
 * PageRank runs as one batch (every space joins it, as fl_batch_add with the
 * space's row_mapping; only an explicit lanes-per-row CSR layout runs
 * alone through fl_execute).  All array arguments have n_spaces entries; d_pagerank[j] /
 * d_minima[j] are sized as for fl_execute (n_raw upper bound is always
 * enough).  out[j].status holds each space's status; the call returns the
 * first error, or FL_ENOCONV if some space did not converge.  The context
 * keeps the batch between calls (empty between calls; freed by fl_destroy),
 * so calls on one context must not overlap. */
fl_status fl_analyze_batch(fl_ctx *ctx, int32_t n_spaces, const fl_space *spaces,
                           const float *const *d_fitness_raw, const fl_neighbourhood *nb,
                           const fl_params *params, double *const *d_pagerank, int32_t *const *d_minima,
                           fl_summary *out);

#ifdef __cplusplus
}
#endif

#endif /* FL_H */
