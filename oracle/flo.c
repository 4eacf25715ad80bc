/*
 * flo.c - FP64 CPU oracle for the fitness-flow-graph (FFG) landscape metric.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this library to check the GPU engine; the engine
 * itself never loads, links or calls it, and the two share no source.
 *
 * It is plain, single-threaded and written to be read against the paper
 * (Schoonhoven, van Werkhoven, Batenburg, "Benchmarking optimization
 * algorithms for auto-tuning GPU kernels"):
 *   - search space X = S_1 x ... x S_n                     (Sec. III-B)
 *   - failed configurations                                (Sec. V)
 *   - Hamming neighbourhood N(x)                           (Sec. III-B, eq. 2)
 *   - adjacent neighbourhood                               (Sec. III-B)
 *   - local minimum                                        (Sec. III-B)
 *   - fitness flow graph, PageRank centrality              (Sec. VII-B)
 *   - p-proportion of centrality C_p                       (Sec. VII-B, eq. 3)
 *   - naive metric: f_opt / f over the local minima        (Sec. VII-A)
 *
 * Readings taken where the paper is silent or ambiguous:
 *   - A configuration is a node iff its fitness is finite and > 0; the caller
 *     marks constraint-violating and failed configurations with +inf / NaN.
 *     A fitness <= 0 or -inf is an error.
 *   - Edge u -> w iff w is a neighbour of u and f(w) < f(u), compared exactly
 *     in float32.  Equal neighbours get no edge.
 *   - Local minimum == sink: no neighbour with strictly lower fitness
 *     (plateau points and isolated nodes count).
 *   - PageRank: the stationary vector r (sum 1) of
 *       G = d*(P + (1/N) 1 s^T) + ((1-d)/N) 1 1^T,
 *     P[w,u] = 1/out_deg(u) for every edge u -> w, s = indicator of sinks,
 *     i.e. damping d with uniform teleport, and the mass of a sink is spread
 *     uniformly over all N nodes.
 *   - L_p = minima m with (double)f(m) <= (1+p)*f_opt, p a fraction.
 *   - Parameter 0 is the most significant mixed-radix digit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define FLO_OK 0
#define FLO_EINVAL (-1)
#define FLO_ENOMEM (-2)
#define FLO_ENOCONV (-4)
#define FLO_EOVERFLOW (-5)

#define FLO_MAX_PARAMS 32

enum { FLO_HAMMING = 0, FLO_ADJACENT = 1 };

typedef struct {
    int n;                          /* number of tunable parameters */
    int neighbourhood;              /* FLO_HAMMING or FLO_ADJACENT */
    int64_t radix[FLO_MAX_PARAMS];  /* |S_i| */
    int64_t stride[FLO_MAX_PARAMS]; /* prod_{j>i} |S_j| */
    int64_t n_raw;                  /* |S_1 x ... x S_n| */

    int64_t N;          /* number of valid points = FFG nodes */
    int64_t *valid_raw; /* node id -> raw index, ascending */
    int64_t *node_of;   /* raw index -> node id, or -1 */
    float *f;           /* fitness per node */
    double f_opt;       /* min fitness, widened exactly */

    int64_t E;          /* number of FFG edges */
    int64_t *out_deg;   /* per node */
    int64_t *in_ptr;    /* CSR over in-edges: sources of w are */
    int64_t *in_src;    /*   in_src[in_ptr[w] .. in_ptr[w+1]) ascending */

    int64_t M;          /* number of local minima */
    int64_t *minima;    /* ascending node ids */
    int64_t plateau_minima; /* minima with an equal-fitness neighbour */
} flo_graph;

static int is_valid(float v) { return isfinite(v) && v > 0.0f; }

/* Compensated (Neumaier) summation: sums over millions of ranks stay exact to
 * a few ulps, so sum(r) = 1 holds to rounding and the L1 residual can fall
 * below 1e-13 (a plain running sum drifts by ~1e-12 at N ~ 1e5). */
typedef struct { double s, c; } flo_sum;

static void sum_add(flo_sum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double sum_get(const flo_sum *a) { return a->s + a->c; }

/* Digits of raw index I: x_i = floor(I / stride_i) mod |S_i|. */
static void digits_of(const flo_graph *g, int64_t I, int64_t *x)
{
    for (int i = 0; i < g->n; ++i)
        x[i] = (I / g->stride[i]) % g->radix[i];
}

/*
 * Valid neighbours of the point with raw index I (Sec. III-B).
 * Hamming: every point that differs from x in exactly one coordinate.
 * Adjacent: as Hamming, but the differing coordinate must hold the value
 * next to x_i in the list S_i (index distance 1, no wrap-around).
 * Points outside X (excluded configurations) are not neighbours, and an
 * excluded index-adjacent value is not skipped over.
 * Writes raw indices to out (room for sum_i |S_i| entries) and returns the count.
 */
static int64_t neighbours_of(const flo_graph *g, int64_t I, int64_t *out)
{
    int64_t x[FLO_MAX_PARAMS];
    int64_t count = 0;
    digits_of(g, I, x);
    for (int i = 0; i < g->n; ++i) {
        for (int64_t a = 0; a < g->radix[i]; ++a) {
            if (a == x[i])
                continue;
            if (g->neighbourhood == FLO_ADJACENT && llabs(a - x[i]) != 1)
                continue;
            int64_t J = I + (a - x[i]) * g->stride[i];
            if (g->node_of[J] >= 0)
                out[count++] = J;
        }
    }
    return count;
}

/* 1 iff node v has a valid neighbour whose fitness equals f(v) exactly. */
static int has_equal_neighbour(const flo_graph *g, int64_t v, int64_t *nb)
{
    int64_t k = neighbours_of(g, g->valid_raw[v], nb);
    for (int64_t j = 0; j < k; ++j)
        if (g->f[g->node_of[nb[j]]] == g->f[v])
            return 1;
    return 0;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

void flo_free(flo_graph *g)
{
    if (!g)
        return;
    free(g->valid_raw);
    free(g->node_of);
    free(g->f);
    free(g->out_deg);
    free(g->in_ptr);
    free(g->in_src);
    free(g->minima);
    free(g);
}

/*
 * Build the search space, the FFG and its local minima.
 * radix[i] = |S_i| >= 1, fitness_raw has prod radix entries in mixed-radix
 * order with parameter 0 most significant.
 */
int flo_build(int n, const int32_t *radix, const float *fitness_raw,
              int neighbourhood, flo_graph **out)
{
    *out = NULL;
    if (n < 1 || n > FLO_MAX_PARAMS)
        return FLO_EINVAL;
    if (neighbourhood != FLO_HAMMING && neighbourhood != FLO_ADJACENT)
        return FLO_EINVAL;
    flo_graph *g = calloc(1, sizeof *g);
    if (!g)
        return FLO_ENOMEM;
    g->n = n;
    g->neighbourhood = neighbourhood;

    /* X = S_1 x ... x S_n: sizes and mixed-radix strides (Sec. III-B). */
    g->n_raw = 1;
    for (int i = 0; i < n; ++i) {
        if (radix[i] < 1) { flo_free(g); return FLO_EINVAL; }
        g->radix[i] = radix[i];
        g->n_raw *= radix[i];
        if (g->n_raw >= ((int64_t)1 << 31)) { flo_free(g); return FLO_EOVERFLOW; }
    }
    for (int i = n - 1; i >= 0; --i)
        g->stride[i] = (i == n - 1) ? 1 : g->stride[i + 1] * g->radix[i + 1];

    /* Valid points, node ids in ascending raw order, f_opt (Sec. VII-B). */
    g->node_of = malloc(sizeof(int64_t) * g->n_raw);
    if (!g->node_of) { flo_free(g); return FLO_ENOMEM; }
    g->N = 0;
    for (int64_t I = 0; I < g->n_raw; ++I) {
        float v = fitness_raw[I];
        if (!isnan(v) && !(v > 0.0f)) { flo_free(g); return FLO_EINVAL; } /* <= 0 or -inf */
        g->node_of[I] = is_valid(v) ? g->N++ : -1;
    }
    if (g->N == 0) { flo_free(g); return FLO_EINVAL; }
    g->valid_raw = malloc(sizeof(int64_t) * g->N);
    g->f = malloc(sizeof(float) * g->N);
    g->out_deg = calloc(g->N, sizeof(int64_t));
    g->in_ptr = calloc(g->N + 1, sizeof(int64_t));
    if (!g->valid_raw || !g->f || !g->out_deg || !g->in_ptr) { flo_free(g); return FLO_ENOMEM; }
    g->f_opt = INFINITY;
    for (int64_t I = 0; I < g->n_raw; ++I) {
        int64_t v = g->node_of[I];
        if (v < 0)
            continue;
        g->valid_raw[v] = I;
        g->f[v] = fitness_raw[I];
        if ((double)g->f[v] < g->f_opt)
            g->f_opt = (double)g->f[v];
    }

    /* FFG (Sec. VII-B): edge u -> w iff w in N(u) and f(w) < f(u).
     * Pass 1 counts out-degrees and in-degrees. */
    int64_t max_nb = 0;
    for (int i = 0; i < n; ++i)
        max_nb += g->radix[i];
    int64_t *nb = malloc(sizeof(int64_t) * (size_t)(max_nb > 0 ? max_nb : 1));
    if (!nb) { flo_free(g); return FLO_ENOMEM; }
    for (int64_t u = 0; u < g->N; ++u) {
        int64_t k = neighbours_of(g, g->valid_raw[u], nb);
        for (int64_t j = 0; j < k; ++j) {
            int64_t w = g->node_of[nb[j]];
            if (g->f[w] < g->f[u]) {
                g->out_deg[u] += 1;
                g->in_ptr[w + 1] += 1;
            }
        }
    }
    for (int64_t w = 0; w < g->N; ++w)
        g->in_ptr[w + 1] += g->in_ptr[w];
    g->E = g->in_ptr[g->N];
    if (g->E >= ((int64_t)1 << 31)) { free(nb); flo_free(g); return FLO_EOVERFLOW; }

    /* Pass 2 fills the in-edge lists, then sorts each by source id. */
    g->in_src = malloc(sizeof(int64_t) * (size_t)(g->E > 0 ? g->E : 1));
    int64_t *fill = malloc(sizeof(int64_t) * g->N);
    if (!g->in_src || !fill) { free(nb); free(fill); flo_free(g); return FLO_ENOMEM; }
    memcpy(fill, g->in_ptr, sizeof(int64_t) * g->N);
    for (int64_t u = 0; u < g->N; ++u) {
        int64_t k = neighbours_of(g, g->valid_raw[u], nb);
        for (int64_t j = 0; j < k; ++j) {
            int64_t w = g->node_of[nb[j]];
            if (g->f[w] < g->f[u])
                g->in_src[fill[w]++] = u;
        }
    }
    free(fill);
    for (int64_t w = 0; w < g->N; ++w)
        qsort(g->in_src + g->in_ptr[w], (size_t)(g->in_ptr[w + 1] - g->in_ptr[w]),
              sizeof(int64_t), cmp_i64);

    /* Local minima = sinks: no neighbour with lower fitness (Sec. III-B). */
    g->M = 0;
    for (int64_t v = 0; v < g->N; ++v)
        g->M += (g->out_deg[v] == 0);
    g->minima = malloc(sizeof(int64_t) * (size_t)(g->M > 0 ? g->M : 1));
    if (!g->minima) { free(nb); flo_free(g); return FLO_ENOMEM; }
    int64_t m = 0;
    for (int64_t v = 0; v < g->N; ++v) {
        if (g->out_deg[v] != 0)
            continue;
        g->minima[m++] = v;
    }

    /* Plateau minima: sinks with a valid neighbour of exactly equal fitness
     * (the points the strict reading of Sec. III-B, "all neighbours worse",
     * would not call minima). */
    g->plateau_minima = 0;
    for (int64_t j = 0; j < g->M; ++j)
        g->plateau_minima += has_equal_neighbour(g, g->minima[j], nb);
    free(nb);
    *out = g;
    return FLO_OK;
}

/* sizes[0..5] = n_raw, N, E, M, plateau minima, max candidate slots K. */
void flo_sizes(const flo_graph *g, int64_t *sizes)
{
    int64_t K = 0;
    for (int i = 0; i < g->n; ++i)
        K += (g->neighbourhood == FLO_ADJACENT) ? (g->radix[i] > 2 ? 2 : g->radix[i] - 1)
                                                : g->radix[i] - 1;
    sizes[0] = g->n_raw;
    sizes[1] = g->N;
    sizes[2] = g->E;
    sizes[3] = g->M;
    sizes[4] = g->plateau_minima;
    sizes[5] = K;
}

double flo_f_opt(const flo_graph *g) { return g->f_opt; }

/* Copy the graph out as int32 arrays (any pointer may be NULL). */
void flo_export(const flo_graph *g, int32_t *valid_raw, int32_t *in_ptr,
                int32_t *in_src, int32_t *out_deg, int32_t *minima, float *f)
{
    for (int64_t v = 0; v < g->N; ++v) {
        if (valid_raw) valid_raw[v] = (int32_t)g->valid_raw[v];
        if (out_deg) out_deg[v] = (int32_t)g->out_deg[v];
        if (f) f[v] = g->f[v];
    }
    if (in_ptr)
        for (int64_t v = 0; v <= g->N; ++v) in_ptr[v] = (int32_t)g->in_ptr[v];
    if (in_src)
        for (int64_t e = 0; e < g->E; ++e) in_src[e] = (int32_t)g->in_src[e];
    if (minima)
        for (int64_t m = 0; m < g->M; ++m) minima[m] = (int32_t)g->minima[m];
}

/* Raw indices of the valid neighbours of node v, any order; returns count. */
int64_t flo_neighbour_list(const flo_graph *g, int64_t v, int32_t *out_raw)
{
    int64_t max_nb = 0;
    for (int i = 0; i < g->n; ++i)
        max_nb += g->radix[i];
    int64_t *nb = malloc(sizeof(int64_t) * (size_t)max_nb);
    if (!nb)
        return FLO_ENOMEM;
    int64_t k = neighbours_of(g, g->valid_raw[v], nb);
    for (int64_t j = 0; j < k; ++j)
        out_raw[j] = (int32_t)nb[j];
    free(nb);
    return k;
}

/*
 * PageRank centrality on the FFG (Sec. VII-B): the dominant right
 * eigenvector of the column-stochastic matrix G above, normalised to sum 1.
 * Power iteration from r = 1/N, renormalised each step, until
 * ||r' - r||_1 <= tol or max_iter steps.  All arithmetic in FP64.
 */
int flo_pagerank(const flo_graph *g, double d, double tol, int64_t max_iter,
                 double *r, int64_t *iterations, double *residual)
{
    if (!(d > 0.0 && d < 1.0))
        return FLO_EINVAL;
    const int64_t N = g->N;
    double *next = malloc(sizeof(double) * N);
    if (!next)
        return FLO_ENOMEM;
    for (int64_t v = 0; v < N; ++v)
        r[v] = 1.0 / (double)N;
    int64_t it = 0;
    double rho = INFINITY;
    while (it < max_iter) {
        flo_sum total_acc = {0, 0}, sink_acc = {0, 0}, next_acc = {0, 0}, rho_acc = {0, 0};
        for (int64_t v = 0; v < N; ++v) {
            sum_add(&total_acc, r[v]);
            if (g->out_deg[v] == 0)
                sum_add(&sink_acc, r[v]);
        }
        double total = sum_get(&total_acc), sink_mass = sum_get(&sink_acc);
        /* (G r)[w] = d * sum_{u->w} r[u]/out_deg(u) + d*sink_mass/N + (1-d)*total/N */
        double spread = (d * sink_mass + (1.0 - d) * total) / (double)N;
        for (int64_t w = 0; w < N; ++w) {
            double acc = 0.0;
            for (int64_t e = g->in_ptr[w]; e < g->in_ptr[w + 1]; ++e) {
                int64_t u = g->in_src[e];
                acc += r[u] / (double)g->out_deg[u];
            }
            next[w] = d * acc + spread;
            sum_add(&next_acc, next[w]);
        }
        double next_total = sum_get(&next_acc);
        for (int64_t v = 0; v < N; ++v) {
            next[v] /= next_total;
            sum_add(&rho_acc, fabs(next[v] - r[v]));
        }
        rho = sum_get(&rho_acc);
        memcpy(r, next, sizeof(double) * N);
        ++it;
        if (rho <= tol)
            break;
    }
    free(next);
    *iterations = it;
    *residual = rho;
    return rho <= tol ? FLO_OK : FLO_ENOCONV;
}

/*
 * Exact PageRank of the FFG without iteration (Sec. VII-B), for damping
 * d in (0, 1].  Both the teleport and the sink term of G are multiples of
 * the all-ones vector, so the stationary vector is r = u / sum(u) with
 * (I - d P) u = 1, i.e. u(w) = 1 + d * sum_{u->w} u(u) / out_deg(u).  Every
 * edge goes from higher to lower fitness, so nodes in order of descending
 * fitness have all their in-neighbours before them: one forward
 * substitution in that order solves the system.  *depth receives the length
 * of the longest path (edges) of the FFG.  At d = 1, u(m) / N for a sink m
 * is the probability that a descent from a uniformly random start, moving
 * to a uniformly random better neighbour until none exists, ends in m.
 */
static const float *g_sort_f;

static int by_fitness_desc(const void *a, const void *b)
{
    float fa = g_sort_f[*(const int64_t *)a], fb = g_sort_f[*(const int64_t *)b];
    if (fa > fb) return -1;
    if (fa < fb) return 1;
    int64_t ia = *(const int64_t *)a, ib = *(const int64_t *)b;
    return (ia > ib) - (ia < ib);
}

int flo_dag_rank(const flo_graph *g, double d, double *r, int64_t *depth)
{
    if (!(d > 0.0 && d <= 1.0))
        return FLO_EINVAL;
    const int64_t N = g->N;
    int64_t *order = malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    int64_t *level = calloc((size_t)(N > 0 ? N : 1), sizeof(int64_t));
    if (!order || !level) { free(order); free(level); return FLO_ENOMEM; }
    for (int64_t v = 0; v < N; ++v)
        order[v] = v;
    g_sort_f = g->f;
    qsort(order, (size_t)N, sizeof(int64_t), by_fitness_desc);
    int64_t deepest = 0;
    for (int64_t j = 0; j < N; ++j) {
        int64_t w = order[j];
        flo_sum acc = {0, 0};
        for (int64_t e = g->in_ptr[w]; e < g->in_ptr[w + 1]; ++e) {
            int64_t u = g->in_src[e];
            sum_add(&acc, r[u] / (double)g->out_deg[u]);
            if (level[u] + 1 > level[w])
                level[w] = level[u] + 1;
        }
        r[w] = 1.0 + d * sum_get(&acc);
        if (level[w] > deepest)
            deepest = level[w];
    }
    flo_sum total = {0, 0};
    for (int64_t v = 0; v < N; ++v)
        sum_add(&total, r[v]);
    double t = sum_get(&total);
    for (int64_t v = 0; v < N; ++v)
        r[v] /= t;
    free(order);
    free(level);
    if (depth)
        *depth = deepest;
    return FLO_OK;
}

/*
 * p-proportion of centrality (Sec. VII-B, eq. 3):
 *   C_p = sum_{x in L_p} c(x) / sum_{x in L} c(x),
 * L the local minima, L_p those with fitness <= (1+p) f_opt.
 * Sums run over the minima in ascending node id, compensated FP64.
 */
double flo_score(const flo_graph *g, const double *c, double p, double *num, double *den)
{
    double threshold = (1.0 + p) * g->f_opt;
    flo_sum near_acc = {0, 0}, all_acc = {0, 0};
    for (int64_t m = 0; m < g->M; ++m) {
        int64_t v = g->minima[m];
        sum_add(&all_acc, c[v]);
        if ((double)g->f[v] <= threshold)
            sum_add(&near_acc, c[v]);
    }
    double s_near = sum_get(&near_acc), s_all = sum_get(&all_acc);
    if (num) *num = s_near;
    if (den) *den = s_all;
    return s_near / s_all;
}

/*
 * Naive landscape metric (Sec. VII-A): for every local minimum m the fraction
 * of optimal fitness it reaches, f_opt / f(m) in (0, 1], FP64 from the
 * float32 fitness values.  ratio[j] (may be NULL) belongs to the j-th
 * minimum in ascending node id.  hist (may be NULL, n_bins >= 1 entries)
 * counts the minima per equal-width bin of [0, 1]: a ratio q falls in bin
 * floor(q * n_bins), and q = 1 in the last bin.
 * Returns FLO_OK, or FLO_EINVAL for n_bins < 1 when hist is given.
 */
int flo_naive(const flo_graph *g, double *ratio, int64_t n_bins, int64_t *hist)
{
    if (hist && n_bins < 1)
        return FLO_EINVAL;
    if (hist)
        for (int64_t b = 0; b < n_bins; ++b)
            hist[b] = 0;
    for (int64_t j = 0; j < g->M; ++j) {
        double q = g->f_opt / (double)g->f[g->minima[j]];
        if (ratio)
            ratio[j] = q;
        if (hist) {
            int64_t b = (int64_t)floor(q * (double)n_bins);
            if (b > n_bins - 1)
                b = n_bins - 1;
            hist[b] += 1;
        }
    }
    return FLO_OK;
}

/*
 * One whole analysis in one call (the steps above, in order): FFG, local
 * minima, PageRank and C_p of one space, host buffers, FP64.
 *   outputs (any may be NULL): pagerank[N], minima[M], valid_raw[N],
 *   row_ptr[N + 1] and col_idx[E] (the in-edge lists, sources ascending);
 *   n_raw-sized buffers always suffice for all but col_idx, which holds
 *   cap_edges entries.
 *   sizes (7 x int64, may be NULL): n_raw, N, E, M, plateau minima,
 *   iterations, K (candidate neighbour slots per node).
 *   stats (5 x double, may be NULL): residual, f_opt, C_p, mass of L_p,
 *   mass of L.
 * Returns FLO_OK; FLO_EINVAL / FLO_ENOMEM / FLO_EOVERFLOW as flo_build and
 * flo_pagerank; FLO_ENOCONV when max_iter was reached (outputs written);
 * FLO_ESIZE when E > cap_edges (sizes written, nothing else).
 */
#define FLO_ESIZE (-6)
int flo_analyze(int n, const int32_t *radix, const float *fitness_raw, int neighbourhood, double damping,
                double p, double tol, int64_t max_iter, double *pagerank, int32_t *minima, int32_t *valid_raw,
                int32_t *row_ptr, int32_t *col_idx, int64_t cap_edges, int64_t *sizes, double *stats)
{
    flo_graph *g = NULL;
    int rc = flo_build(n, radix, fitness_raw, neighbourhood, &g);
    if (rc != FLO_OK)
        return rc;
    int64_t s6[6];
    flo_sizes(g, s6);
    if (sizes) {
        for (int j = 0; j < 5; ++j)
            sizes[j] = s6[j];
        sizes[5] = 0;
        sizes[6] = s6[5];
    }
    if (col_idx && g->E > cap_edges) {
        flo_free(g);
        return FLO_ESIZE;
    }
    double *r = malloc(sizeof(double) * (size_t)(g->N > 0 ? g->N : 1));
    if (!r) {
        flo_free(g);
        return FLO_ENOMEM;
    }
    int64_t iterations = 0;
    double residual = 0.0;
    rc = flo_pagerank(g, damping, tol, max_iter, r, &iterations, &residual);
    if (rc == FLO_OK || rc == FLO_ENOCONV) {
        double num = 0.0, den = 0.0;
        const double score = flo_score(g, r, p, &num, &den);
        flo_export(g, valid_raw, row_ptr, col_idx, NULL, minima, NULL);
        if (pagerank)
            memcpy(pagerank, r, sizeof(double) * (size_t)g->N);
        if (sizes)
            sizes[5] = iterations;
        if (stats) {
            stats[0] = residual;
            stats[1] = g->f_opt;
            stats[2] = score;
            stats[3] = num;
            stats[4] = den;
        }
    }
    free(r);
    flo_free(g);
    return rc;
}
