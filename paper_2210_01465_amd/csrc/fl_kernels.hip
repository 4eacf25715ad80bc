// fl_kernels.hip - gfx950 kernels of the fitness-flow-graph engine.
//
// Steps (paper: Schoonhoven et al., "Benchmarking optimization algorithms for
// auto-tuning GPU kernels"):
//   compaction      valid points of X = S_1 x ... x S_n              (Sec. III-B, Sec. V)
//   degree count    neighbours (eq. 2 / adjacent), edges to strictly
//                   better neighbours                                 (Sec. VII-B)
//   scan + fill     CSR over in-edges, local minima = sinks           (Sec. III-B, Sec. VII-B)
//   power iteration PageRank centrality of the FFG                    (Sec. VII-B)
//   score           p-proportion of centrality C_p                   (Sec. VII-B, eq. 3)
//
// All of it is integer or memory-bound work: no dense contraction exists on
// this path, so nothing here uses MFMA.  The kernels are written for 64-wide
// waves and 256-thread workgroups; the iteration kernel maps contiguous row
// ranges to each XCD so that the x gathers of one row range stay in one L2.
#include <math.h>

#include "fl_internal.h"

namespace fl {
namespace {

__device__ __forceinline__ bool valid_fitness(float f) { return f > 0.0f && f < INFINITY; }
// fitness <= 0 or -inf (NaN and +inf mark excluded configurations)
__device__ __forceinline__ bool bad_fitness(float f) { return !(f != f) && !(f > 0.0f); }

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

__device__ __forceinline__ float wave_min(float x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fminf(x, __shfl_xor(x, o, 64));
    return x;
}

// Sum over the workgroup; the result is valid in every thread.  The fixed
// shape of the tree makes floating-point sums deterministic.
template <typename T>
__device__ T block_sum(T v) {
    __shared__ T part[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_sum(v);
    if (lane == 0) part[wid] = v;
    __syncthreads();
    T t = part[0];
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w) t += part[w];
    __syncthreads();
    return t;
}

__device__ float block_min(float v) {
    __shared__ float part[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    v = wave_min(v);
    if (lane == 0) part[wid] = v;
    __syncthreads();
    float t = part[0];
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w) t = fminf(t, part[w]);
    __syncthreads();
    return t;
}

// Exclusive prefix sum over the workgroup; *total receives the sum.
template <typename T>
__device__ T block_excl_scan(T v, T *total) {
    __shared__ T part[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) part[wid] = incl;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        T s = part[w];
        off += (w < wid) ? s : T(0);
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

// Single-workgroup exclusive scan of a tile-count array of any length, in
// chunks of kBlock*8 with a running carry.  Returns the grand total.
template <typename T>
__device__ T scan_tiles(const T *in, T *out, int n_tiles) {
    T carry = 0;
    for (int base = 0; base < n_tiles; base += kBlock * 8) {
        T v[8];
        T s = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int idx = base + threadIdx.x * 8 + j;
            v[j] = idx < n_tiles ? in[idx] : T(0);
            s += v[j];
        }
        T tot;
        T run = carry + block_excl_scan(s, &tot);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int idx = base + threadIdx.x * 8 + j;
            if (idx < n_tiles) out[idx] = run;
            run += v[j];
        }
        carry += tot;
    }
    return carry;
}

// ---------------------------------------------------------------------------
// Compaction: valid points in ascending raw order (Sec. III-B; failed and
// constraint-violating configurations are excluded, Sec. V), f_opt.

__global__ __launch_bounds__(kBlock) void k_compact_count(const float *__restrict__ fit, int32_t n_raw,
                                                          int32_t *__restrict__ tile_cnt,
                                                          float *__restrict__ tile_min,
                                                          int32_t *__restrict__ tile_bad) {
    const int64_t base = (int64_t)blockIdx.x * kCompactTile;
    int32_t cnt = 0, bad = 0;
    float mn = INFINITY;
#pragma unroll
    for (int j = 0; j < kCompactItems; ++j) {
        const int64_t i = base + j * kBlock + threadIdx.x;
        if (i < n_raw) {
            const float f = fit[i];
            const bool v = valid_fitness(f);
            cnt += v;
            bad += bad_fitness(f);
            if (v) mn = fminf(mn, f);
        }
    }
    cnt = block_sum(cnt);
    bad = block_sum(bad);
    mn = block_min(mn);
    if (threadIdx.x == 0) {
        tile_cnt[blockIdx.x] = cnt;
        tile_bad[blockIdx.x] = bad;
        tile_min[blockIdx.x] = mn;
    }
}

__global__ __launch_bounds__(kBlock) void k_compact_scan(const int32_t *__restrict__ tile_cnt,
                                                         const float *__restrict__ tile_min,
                                                         const int32_t *__restrict__ tile_bad,
                                                         int32_t n_tiles, int32_t *__restrict__ tile_off,
                                                         BuildSizes *__restrict__ sizes) {
    const int32_t n_valid = scan_tiles(tile_cnt, tile_off, n_tiles);
    int32_t bad = 0;
    float mn = INFINITY;
    for (int t = threadIdx.x; t < n_tiles; t += kBlock) {
        bad += tile_bad[t];
        mn = fminf(mn, tile_min[t]);
    }
    bad = block_sum(bad);
    mn = block_min(mn);
    if (threadIdx.x == 0) {
        sizes->n_valid = n_valid;
        sizes->n_bad = bad;
        sizes->f_opt = mn;
    }
}

__global__ __launch_bounds__(kBlock) void k_compact_write(const float *__restrict__ fit, int32_t n_raw,
                                                          const int32_t *__restrict__ tile_off,
                                                          int32_t *__restrict__ remap,
                                                          int32_t *__restrict__ valid_raw,
                                                          float *__restrict__ fit_c) {
    // blocked: thread t owns raw indices base + t*8 .. base + t*8 + 7
    const int64_t base = (int64_t)blockIdx.x * kCompactTile + (int64_t)threadIdx.x * kCompactItems;
    float f[kCompactItems];
    int32_t s = 0;
#pragma unroll
    for (int j = 0; j < kCompactItems; ++j) {
        const int64_t i = base + j;
        f[j] = i < n_raw ? fit[i] : NAN;
        s += valid_fitness(f[j]);
    }
    int32_t tot;
    int32_t id = tile_off[blockIdx.x] + block_excl_scan(s, &tot);
#pragma unroll
    for (int j = 0; j < kCompactItems; ++j) {
        const int64_t i = base + j;
        if (i >= n_raw) break;
        if (valid_fitness(f[j])) {
            remap[i] = id;
            valid_raw[id] = (int32_t)i;
            fit_c[id] = f[j];
            ++id;
        } else {
            remap[i] = -1;
        }
    }
}

// ---------------------------------------------------------------------------
// FFG degrees (Sec. VII-B): for node v with raw index i and digits x, every
// candidate neighbour is c = i + (a - x_k) * stride_k (eq. 2: one parameter
// changed; adjacent: a = x_k +- 1 inside the list).  in_deg counts valid
// neighbours with strictly higher fitness (edges into v), out_deg those with
// strictly lower fitness (edges out of v).  One thread per node: the wave's
// 64 nodes are consecutive valid points, so each candidate slot is a
// near-contiguous gather.

template <bool ADJ>
__global__ __launch_bounds__(kBlock) void k_degree(SpaceDesc sp, const float *__restrict__ fit,
                                                   const int32_t *__restrict__ valid_raw, int32_t n,
                                                   int32_t *__restrict__ in_deg,
                                                   int32_t *__restrict__ out_deg,
                                                   int64_t *__restrict__ tile_e,
                                                   int32_t *__restrict__ tile_m) {
    const int32_t v = blockIdx.x * kBlock + threadIdx.x;
    int32_t din = 0, dout = 0;
    if (v < n) {
        const uint32_t i = (uint32_t)valid_raw[v];
        const float fv = fit[i];
        for (int k = 0; k < sp.n; ++k) {
            const uint32_t r = (uint32_t)sp.radix[k], st = (uint32_t)sp.stride[k];
            const uint32_t xk = (i / st) % r;
            const uint32_t row = i - xk * st;
            if (ADJ) {
                if (xk > 0) {
                    const float fc = fit[row + (xk - 1) * st];
                    din += (fc > fv) & (fc < INFINITY);
                    dout += (fc < fv);
                }
                if (xk + 1 < r) {
                    const float fc = fit[row + (xk + 1) * st];
                    din += (fc > fv) & (fc < INFINITY);
                    dout += (fc < fv);
                }
            } else {
                for (uint32_t a = 0; a < r; ++a) {
                    if (a == xk) continue;
                    const float fc = fit[row + a * st];
                    din += (fc > fv) & (fc < INFINITY);
                    dout += (fc < fv);
                }
            }
        }
        in_deg[v] = din;
        out_deg[v] = dout;
    }
    const int64_t te = block_sum((int64_t)din);
    const int32_t tm = block_sum((int32_t)(v < n && dout == 0));
    if (threadIdx.x == 0) {
        tile_e[blockIdx.x] = te;
        tile_m[blockIdx.x] = tm;
    }
}

__global__ __launch_bounds__(kBlock) void k_degree_scan(const int64_t *__restrict__ tile_e,
                                                        const int32_t *__restrict__ tile_m,
                                                        int32_t n_tiles, int64_t *__restrict__ tile_eoff,
                                                        int32_t *__restrict__ tile_moff,
                                                        BuildSizes *__restrict__ sizes) {
    const int64_t e = scan_tiles(tile_e, tile_eoff, n_tiles);
    const int32_t m = scan_tiles(tile_m, tile_moff, n_tiles);
    if (threadIdx.x == 0) {
        sizes->n_edges = e;
        sizes->n_minima = m;
    }
}

// CSR fill: row_ptr by a workgroup scan of in_deg plus the tile offset, the
// minima (sinks) by a scan of the sink flags, then the sources of every
// in-edge in ascending raw (= node id) order.  Ascending order of
// c = i + (a - x_k) * stride_k is: below i, parameters 0..n-1 with a rising
// from 0 to x_k - 1; above i, parameters n-1..0 with a rising from x_k + 1.

template <bool ADJ>
__device__ __forceinline__ void fill_slot(const float *__restrict__ fit, const int32_t *__restrict__ remap,
                                          uint32_t c, float fv, int32_t *__restrict__ col_idx,
                                          int32_t &pos, int32_t end) {
    const float fc = fit[c];
    if ((fc > fv) & (fc < INFINITY)) {
        if (pos < end) col_idx[pos] = remap[c];
        ++pos;
    }
}

template <bool ADJ>
__global__ __launch_bounds__(kBlock) void k_fill(SpaceDesc sp, const float *__restrict__ fit,
                                                 const int32_t *__restrict__ valid_raw,
                                                 const int32_t *__restrict__ remap, int32_t n,
                                                 int32_t n_edges, const int32_t *__restrict__ in_deg,
                                                 const int32_t *__restrict__ out_deg,
                                                 const int64_t *__restrict__ tile_eoff,
                                                 const int32_t *__restrict__ tile_moff,
                                                 int32_t *__restrict__ row_ptr,
                                                 int32_t *__restrict__ col_idx,
                                                 int32_t *__restrict__ minima) {
    const int32_t v = blockIdx.x * kBlock + threadIdx.x;
    const int32_t din = v < n ? in_deg[v] : 0;
    const int32_t sink = (v < n && out_deg[v] == 0) ? 1 : 0;
    int32_t tot;
    const int32_t e_off = (int32_t)tile_eoff[blockIdx.x] + block_excl_scan(din, &tot);
    const int32_t m_off = tile_moff[blockIdx.x] + block_excl_scan(sink, &tot);
    if (v >= n) return;
    row_ptr[v] = e_off;
    if (v == n - 1) row_ptr[n] = n_edges;
    if (sink) minima[m_off] = v;
    if (din == 0) return;
    const uint32_t i = (uint32_t)valid_raw[v];
    const float fv = fit[i];
    const int32_t end = e_off + din;
    int32_t pos = e_off;
    for (int k = 0; k < sp.n; ++k) {  // below i
        const uint32_t r = (uint32_t)sp.radix[k], st = (uint32_t)sp.stride[k];
        const uint32_t xk = (i / st) % r;
        const uint32_t row = i - xk * st;
        if (ADJ) {
            if (xk > 0) fill_slot<ADJ>(fit, remap, row + (xk - 1) * st, fv, col_idx, pos, end);
        } else {
            for (uint32_t a = 0; a < xk; ++a) fill_slot<ADJ>(fit, remap, row + a * st, fv, col_idx, pos, end);
        }
    }
    for (int k = sp.n - 1; k >= 0; --k) {  // above i
        const uint32_t r = (uint32_t)sp.radix[k], st = (uint32_t)sp.stride[k];
        const uint32_t xk = (i / st) % r;
        const uint32_t row = i - xk * st;
        if (ADJ) {
            if (xk + 1 < r) fill_slot<ADJ>(fit, remap, row + (xk + 1) * st, fv, col_idx, pos, end);
        } else {
            for (uint32_t a = xk + 1; a < r; ++a) fill_slot<ADJ>(fit, remap, row + a * st, fv, col_idx, pos, end);
        }
    }
}

// ---------------------------------------------------------------------------
// PageRank power iteration (Sec. VII-B) with damping d, uniform teleport and
// sink mass spread uniformly:
//   r'[w] = d * sum_{u->w} r[u]/out_deg(u) + (d * sum_{sinks} r + 1 - d) / N.
// Stored iterate y_k = r_k up to s_k = 1/sum(y_k); x_k = y_k/out_deg.  The
// edge sum is FP32; the per-node affine update, the residual
// ||r_{k+1} - r_k||_1, the renormalisation and the sink mass are FP64.  Each
// workgroup writes FP64 partial sums; the last one to finish (ticket) reduces
// them in a fixed order and sets s, c and the stop flag for the next launch.

__device__ bool elect_last(uint32_t *ticket) {
    __shared__ bool last;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

__device__ void pr_finish(const PrArgs &a, bool first) {
    const int g = gridDim.x;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int b = threadIdx.x; b < g; b += kBlock) {
        s0 += __hip_atomic_load(&a.partials[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s1 += __hip_atomic_load(&a.partials[g + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s2 += __hip_atomic_load(&a.partials[2 * g + b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    s0 = block_sum(s0);
    s1 = block_sum(s1);
    s2 = block_sum(s2);
    if (threadIdx.x == 0) {
        PrState *st = a.st;
        const double sigma = s0, sink = s2;
        const double s = 1.0 / sigma;
        st->sigma = sigma;
        st->sink = sink;
        st->s = s;
        st->c = (a.d * sink * s + (1.0 - a.d)) / (double)a.n;
        if (!first) {
            st->resid_prev = st->resid;
            st->resid = s1;
            st->k += 1;
            st->worked += 1;
            if (s1 < a.tol)
                st->done = 1;
            else if (st->k >= a.max_iter)
                st->done = 2;
        }
        st->ticket = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_pr_init(PrArgs a) {
    const float y0 = (float)(1.0 / (double)a.n);
    double ps = 0.0, pk = 0.0;
    for (int32_t v = blockIdx.x * kBlock + threadIdx.x; v < a.n; v += gridDim.x * kBlock) {
        const int32_t deg = a.out_deg[v];
        a.y[0][v] = y0;
        a.x[0][v] = deg > 0 ? y0 / (float)deg : 0.0f;
        ps += (double)y0;
        if (deg == 0) pk += (double)y0;
    }
    ps = block_sum(ps);
    pk = block_sum(pk);
    const int g = gridDim.x;
    if (threadIdx.x == 0) {
        a.partials[blockIdx.x] = ps;
        a.partials[g + blockIdx.x] = 0.0;
        a.partials[2 * g + blockIdx.x] = pk;
    }
    if (elect_last(&a.st->ticket)) pr_finish(a, true);
}

// L lanes per row: the lanes of a row read consecutive col_idx entries and
// reduce with cross-lane shuffles.  The grid is persistent (a multiple of 8
// workgroups); workgroup b is dealt to XCD b % 8 and gets logical id
// (b % 8) * (G/8) + b / 8, and logical ids own contiguous runs of rows, so
// every XCD sweeps one contiguous eighth of the rows.
template <int L>
__global__ __launch_bounds__(kBlock) void k_pr_iter(PrArgs a) {
    const PrState *st = a.st;
    if (st->done) return;
    const int32_t k = st->k;
    const float *__restrict__ y_in = a.y[k & 1];
    const float *__restrict__ x_in = a.x[k & 1];
    float *__restrict__ y_out = a.y[(k + 1) & 1];
    float *__restrict__ x_out = a.x[(k + 1) & 1];
    const int32_t *__restrict__ row_ptr = a.row_ptr;
    const int32_t *__restrict__ col_idx = a.col_idx;
    const double s = st->s, c = st->c;
    const double sd = s * a.d;

    const int g = gridDim.x;
    const int lb = (blockIdx.x % kXcds) * (g / kXcds) + blockIdx.x / kXcds;
    constexpr int kRows = kBlock / L;
    const int32_t n_groups = (a.n + kRows - 1) / kRows;
    const int32_t chunk = (n_groups + g - 1) / g;
    const int32_t g0 = lb * chunk;
    const int32_t g1 = min(g0 + chunk, n_groups);
    const int lane = threadIdx.x % L;
    const int sub = threadIdx.x / L;

    double ps = 0.0, pr = 0.0, pk = 0.0;
    for (int32_t grp = g0; grp < g1; ++grp) {
        const int32_t v = grp * kRows + sub;
        float acc = 0.0f;
        if (v < a.n) {
            const int32_t e1 = row_ptr[v + 1];
            for (int32_t e = row_ptr[v] + lane; e < e1; e += L) acc += x_in[col_idx[e]];
        }
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0 && v < a.n) {
            const float yf = (float)(sd * (double)acc + c);
            const int32_t deg = a.out_deg[v];
            y_out[v] = yf;
            x_out[v] = deg > 0 ? yf / (float)deg : 0.0f;
            ps += (double)yf;
            pr += fabs((double)yf - s * (double)y_in[v]);
            if (deg == 0) pk += (double)yf;
        }
    }
    ps = block_sum(ps);
    pr = block_sum(pr);
    pk = block_sum(pk);
    if (threadIdx.x == 0) {
        a.partials[blockIdx.x] = ps;
        a.partials[g + blockIdx.x] = pr;
        a.partials[2 * g + blockIdx.x] = pk;
    }
    if (elect_last(&a.st->ticket)) pr_finish(a, false);
}

__global__ __launch_bounds__(kBlock) void k_pr_output(PrArgs a, double *__restrict__ pagerank) {
    const PrState *st = a.st;
    const float *__restrict__ y = a.y[st->k & 1];
    const double s = st->s;
    for (int32_t v = blockIdx.x * kBlock + threadIdx.x; v < a.n; v += gridDim.x * kBlock)
        pagerank[v] = (double)y[v] * s;
}

// C_p (Sec. VII-B, eq. 3): FP64 sums of the ranks over all minima and over
// those with (double) f <= (1+p) f_opt.  One workgroup.
__global__ __launch_bounds__(kBlock) void k_score(const double *__restrict__ pagerank,
                                                  const int32_t *__restrict__ minima, int32_t m,
                                                  const float *__restrict__ fit_c, double threshold,
                                                  PrState *__restrict__ st) {
    double num = 0.0, den = 0.0;
    for (int32_t j = threadIdx.x; j < m; j += kBlock) {
        const int32_t v = minima[j];
        const double r = pagerank[v];
        den += r;
        if ((double)fit_c[v] <= threshold) num += r;
    }
    num = block_sum(num);
    den = block_sum(den);
    if (threadIdx.x == 0) {
        st->score_num = num;
        st->score_den = den;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.

hipError_t launch_compact(const float *fit, int32_t n_raw, int32_t *tile_cnt, float *tile_min,
                          int32_t *tile_bad, int32_t *tile_off, int32_t *remap,
                          int32_t *valid_raw, float *fit_c, BuildSizes *sizes,
                          hipStream_t stream) {
    const int32_t tiles = (n_raw + kCompactTile - 1) / kCompactTile;
    hipLaunchKernelGGL(k_compact_count, dim3(tiles), dim3(kBlock), 0, stream, fit, n_raw, tile_cnt,
                       tile_min, tile_bad);
    hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(kBlock), 0, stream, tile_cnt, tile_min,
                       tile_bad, tiles, tile_off, sizes);
    hipLaunchKernelGGL(k_compact_write, dim3(tiles), dim3(kBlock), 0, stream, fit, n_raw, tile_off,
                       remap, valid_raw, fit_c);
    return hipGetLastError();
}

hipError_t launch_degree(const SpaceDesc &sp, int adjacent, const float *fit,
                         const int32_t *valid_raw, int32_t n, int32_t *in_deg, int32_t *out_deg,
                         int64_t *tile_e, int32_t *tile_m, int64_t *tile_eoff,
                         int32_t *tile_moff, BuildSizes *sizes, hipStream_t stream) {
    const int32_t tiles = (n + kBlock - 1) / kBlock;
    if (adjacent)
        hipLaunchKernelGGL(k_degree<true>, dim3(tiles), dim3(kBlock), 0, stream, sp, fit, valid_raw,
                           n, in_deg, out_deg, tile_e, tile_m);
    else
        hipLaunchKernelGGL(k_degree<false>, dim3(tiles), dim3(kBlock), 0, stream, sp, fit, valid_raw,
                           n, in_deg, out_deg, tile_e, tile_m);
    hipLaunchKernelGGL(k_degree_scan, dim3(1), dim3(kBlock), 0, stream, tile_e, tile_m, tiles,
                       tile_eoff, tile_moff, sizes);
    return hipGetLastError();
}

hipError_t launch_fill(const SpaceDesc &sp, int adjacent, const float *fit,
                       const int32_t *valid_raw, const int32_t *remap, int32_t n, int32_t n_edges,
                       const int32_t *in_deg, const int32_t *out_deg, const int64_t *tile_eoff,
                       const int32_t *tile_moff, int32_t *row_ptr, int32_t *col_idx,
                       int32_t *minima, hipStream_t stream) {
    const int32_t tiles = (n + kBlock - 1) / kBlock;
    if (adjacent)
        hipLaunchKernelGGL(k_fill<true>, dim3(tiles), dim3(kBlock), 0, stream, sp, fit, valid_raw,
                           remap, n, n_edges, in_deg, out_deg, tile_eoff, tile_moff, row_ptr,
                           col_idx, minima);
    else
        hipLaunchKernelGGL(k_fill<false>, dim3(tiles), dim3(kBlock), 0, stream, sp, fit, valid_raw,
                           remap, n, n_edges, in_deg, out_deg, tile_eoff, tile_moff, row_ptr,
                           col_idx, minima);
    return hipGetLastError();
}

hipError_t launch_pr_init(const PrArgs &a, int grid, hipStream_t stream) {
    hipLaunchKernelGGL(k_pr_init, dim3(grid), dim3(kBlock), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_pr_iter(const PrArgs &a, int lanes, int grid, hipStream_t stream) {
    switch (lanes) {
        case 1: hipLaunchKernelGGL(k_pr_iter<1>, dim3(grid), dim3(kBlock), 0, stream, a); break;
        case 2: hipLaunchKernelGGL(k_pr_iter<2>, dim3(grid), dim3(kBlock), 0, stream, a); break;
        case 4: hipLaunchKernelGGL(k_pr_iter<4>, dim3(grid), dim3(kBlock), 0, stream, a); break;
        case 8: hipLaunchKernelGGL(k_pr_iter<8>, dim3(grid), dim3(kBlock), 0, stream, a); break;
        case 16: hipLaunchKernelGGL(k_pr_iter<16>, dim3(grid), dim3(kBlock), 0, stream, a); break;
        case 32: hipLaunchKernelGGL(k_pr_iter<32>, dim3(grid), dim3(kBlock), 0, stream, a); break;
        case 64: hipLaunchKernelGGL(k_pr_iter<64>, dim3(grid), dim3(kBlock), 0, stream, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pr_output(const PrArgs &a, double *pagerank, hipStream_t stream) {
    const int grid = (int)std::min<int64_t>(((int64_t)a.n + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_pr_output, dim3(grid), dim3(kBlock), 0, stream, a, pagerank);
    return hipGetLastError();
}

hipError_t launch_score(const double *pagerank, const int32_t *minima, int32_t m,
                        const float *fit_c, double threshold, PrState *st, hipStream_t stream) {
    hipLaunchKernelGGL(k_score, dim3(1), dim3(kBlock), 0, stream, pagerank, minima, m, fit_c,
                       threshold, st);
    return hipGetLastError();
}

}  // namespace fl
