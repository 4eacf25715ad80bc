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
// No step is a dense contraction, so nothing here uses MFMA: every kernel is
// bound by memory traffic.  The space is mixed-radix, so the neighbours of a
// node sit at fixed offsets in raw-index space.  The node kernels therefore
// run one node per lane with the 64 lanes of a wave on consecutive valid
// points, and walk the candidate slots in the same order in every lane: each
// slot becomes one near-contiguous gather for the whole wave, and the loads of
// kBatch slots are issued back to back before any of them is used.
#include <math.h>

#include <algorithm>

#include "fl_internal.h"

namespace fl {
namespace {

__device__ __forceinline__ bool valid_fitness(float f) { return f > 0.0f && f < INFINITY; }
// fitness <= 0 or -inf (NaN and +inf mark excluded configurations)
__device__ __forceinline__ bool bad_fitness(float f) { return !(f != f) && !(f > 0.0f); }

// Pointer into the constant address space: memory no kernel of the launch
// writes.  Uniform loads through it may go through the scalar unit even after
// the kernel has stored elsewhere, which keeps the slot offsets and presence
// words in SGPRs instead of a VGPR per value.
template <typename T>
using const_ptr = const __attribute__((address_space(4))) T *;
template <typename T>
__device__ __forceinline__ const_ptr<T> to_const(const T *p) {
    return (const_ptr<T>)p;
}

// The first (here: only) argument of a kernel, in place in the kernel-argument
// segment: explicit arguments start at its offset 0.
template <class T>
__device__ __forceinline__ const_ptr<T> kernel_arg() {
    return (const_ptr<T>)__builtin_amdgcn_kernarg_segment_ptr();
}

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
// Node records and candidate slots.

// Node records: W 64-bit words; in-edge bits first, then out_deg in bits
// 24..31 and the raw index in bits 32..63 of the last word.
template <int W>
struct Record {
    uint64_t w[W];
    __device__ __forceinline__ uint32_t word32(int b) const {  // b compile-time after unrolling
        return (b & 1) ? (uint32_t)(w[b >> 1] >> 32) : (uint32_t)w[b >> 1];
    }
    __device__ __forceinline__ int32_t raw() const { return (int32_t)(w[W - 1] >> 32); }
    __device__ __forceinline__ int32_t out_deg() const { return (int32_t)((w[W - 1] >> 24) & 0xffu); }
};

// Slot bits of batch b (slots 32b .. 32b+31) that name real slots: the last
// record word also carries out_deg and the raw index above slot k.
__device__ __forceinline__ uint32_t batch_mask(int b, int k) {
    const int left = k - 32 * b;
    return left >= 32 ? ~0u : (left <= 0 ? 0u : (1u << left) - 1u);
}

template <int W>
__device__ __forceinline__ Record<W> load_record(const uint64_t *__restrict__ rec, int32_t v) {
    Record<W> r;
    const uint64_t *p = rec + (int64_t)v * W;
    if (W % 2 == 0) {
#pragma unroll
        for (int q = 0; q < W; q += 2) {
            const ulonglong2 t = *reinterpret_cast<const ulonglong2 *>(p + q);
            r.w[q] = t.x;
            r.w[q + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < W; ++q) r.w[q] = p[q];
    }
    return r;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x |= (uint32_t)__shfl_xor((int)x, o, 64);
    return x;
}

// Number of set bits of the record's in-edge mask below slot s (compile-time
// word index after unrolling).
template <int W>
__device__ __forceinline__ int bits_below(const Record<W> &r, int s) {
    int c = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) {
        const int lo = q * 64;
        if (s >= lo + 64)
            c += __popcll(r.w[q]);
        else if (s > lo)
            c += __popcll(r.w[q] & ((1ull << (s - lo)) - 1ull));
    }
    return c;
}

// ---------------------------------------------------------------------------
// Compaction: valid points in ascending raw order (Sec. III-B; failed and
// constraint-violating configurations are excluded, Sec. V), f_opt.

__device__ __forceinline__ void compact_count(const float *__restrict__ fit, int32_t n_raw, int32_t tile,
                                              int32_t *__restrict__ tile_cnt, float *__restrict__ tile_min,
                                              int32_t *__restrict__ tile_bad) {
    const int64_t base = (int64_t)tile * kCompactTile;
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
        tile_cnt[tile] = cnt;
        tile_bad[tile] = bad;
        tile_min[tile] = mn;
    }
}

__device__ __forceinline__ void compact_scan(const int32_t *__restrict__ tile_cnt,
                                             const float *__restrict__ tile_min,
                                             const int32_t *__restrict__ tile_bad, int32_t n_tiles,
                                             int32_t *__restrict__ tile_off, BuildSizes *__restrict__ sizes) {
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
        sizes->n_plateau = 0;   // counted by the degree pass
    }
}

__device__ __forceinline__ void compact_write(const float *__restrict__ fit, int32_t n_raw, int32_t tile,
                                              const int32_t *__restrict__ tile_off, int32_t *__restrict__ remap,
                                              int32_t *__restrict__ valid_raw, float *__restrict__ fit_c) {
    // blocked: thread t owns raw indices base + t*8 .. base + t*8 + 7
    const int64_t base = (int64_t)tile * kCompactTile + (int64_t)threadIdx.x * kCompactItems;
    float f[kCompactItems];
    int32_t s = 0;
#pragma unroll
    for (int j = 0; j < kCompactItems; ++j) {
        const int64_t i = base + j;
        f[j] = i < n_raw ? fit[i] : NAN;
        s += valid_fitness(f[j]);
    }
    int32_t tot;
    int32_t id = tile_off[tile] + block_excl_scan(s, &tot);
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

// Compaction of one space in two passes without a scan kernel.  The first
// pass counts each tile's valid points (and its minimum and bad values); in
// the second, tile t sums the counts of tiles 0 .. t-1 itself (a few KB
// from L2, one round of loads), so no tile waits for another, and writes
// its part of the outputs: remap in place, the compacted node map and
// fitness staged in LDS and stored coalesced.  The last tile also writes
// the totals (n_valid, f_opt, the bad count).  Tiles of kSingleTile raw
// configurations, 16 per thread, loaded as float4 when fit is 16-byte
// aligned (VEC).
//
// A single pass with a decoupled look-back (Merrill and Garland 2016:
// publish the tile's count, walk back over the predecessors' published
// words to the first inclusive prefix) measured 50 us at the large workload
// with a 64-wide walk and 39 us with a 256-wide one, against the 18-20 us
// of these two passes: with every tile running at once, few prefixes are
// out when the walks start, and each round is one device-scope load.

template <bool VEC>
__device__ __forceinline__ void load_tile_values(const float *__restrict__ fit, int32_t n_raw, int64_t base,
                                                 int64_t step, float (&f)[kSingleItems]) {
    // value j of the thread: raw index base + (j / 4) * step + j % 4
#pragma unroll
    for (int q = 0; q < kSingleItems / 4; ++q) {
        const int64_t i = base + q * step;
        if (VEC && i + 4 <= n_raw) {
            const float4 a = *reinterpret_cast<const float4 *>(fit + i);
            f[4 * q] = a.x;
            f[4 * q + 1] = a.y;
            f[4 * q + 2] = a.z;
            f[4 * q + 3] = a.w;
        } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) f[4 * q + e] = i + e < n_raw ? fit[i + e] : NAN;
        }
    }
}

template <bool VEC>
__global__ __launch_bounds__(kBlock) void k_compact_tiles(const float *__restrict__ fit, int32_t n_raw,
                                                          int32_t *__restrict__ tile_cnt,
                                                          float *__restrict__ tile_min,
                                                          int32_t *__restrict__ tile_bad) {
    // strided: thread t reads 4 consecutive values at base + 4t + 1024 q
    float f[kSingleItems];
    load_tile_values<VEC>(fit, n_raw, (int64_t)blockIdx.x * kSingleTile + 4 * threadIdx.x, 4 * kBlock, f);
    int32_t cnt = 0, bad = 0;
    float mn = INFINITY;
#pragma unroll
    for (int j = 0; j < kSingleItems; ++j) {
        const bool v = valid_fitness(f[j]);
        cnt += v;
        bad += bad_fitness(f[j]);
        if (v) mn = fminf(mn, f[j]);
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

template <bool VEC>
__global__ __launch_bounds__(kBlock) void k_compact_place(const float *__restrict__ fit, int32_t n_raw,
                                                          int32_t n_tiles, const int32_t *__restrict__ tile_cnt,
                                                          const float *__restrict__ tile_min,
                                                          const int32_t *__restrict__ tile_bad,
                                                          int32_t *__restrict__ remap,
                                                          int32_t *__restrict__ valid_raw,
                                                          float *__restrict__ fit_c,
                                                          BuildSizes *__restrict__ sizes) {
    __shared__ int32_t st_raw[kSingleTile];
    __shared__ float st_fit[kSingleTile];
    const int32_t tile = blockIdx.x;
    const bool last = tile == n_tiles - 1;
    // the tile's first output slot: the counts of the tiles before it (the
    // last tile sums them all, and the bad counts and minima with them)
    int32_t before = 0, bad = 0;
    float mn = INFINITY;
    const int32_t upto = last ? n_tiles : tile;
    for (int32_t u = threadIdx.x; u < upto; u += kBlock) {
        const int32_t c = tile_cnt[u];
        if (u < tile) before += c;
        if (last) {
            bad += tile_bad[u];
            mn = fminf(mn, tile_min[u]);
        }
    }
    const int32_t excl = block_sum(before);
    // blocked: thread t owns raw indices base .. base + 15
    const int64_t base = (int64_t)tile * kSingleTile + (int64_t)threadIdx.x * kSingleItems;
    float f[kSingleItems];
    load_tile_values<VEC>(fit, n_raw, base, 4, f);
    int32_t cnt = 0;
#pragma unroll
    for (int j = 0; j < kSingleItems; ++j) cnt += valid_fitness(f[j]);
    int32_t tot;
    const int32_t local = block_excl_scan(cnt, &tot);
    if (last) {
        bad = block_sum(bad);
        mn = block_min(mn);
        if (threadIdx.x == 0) {
            sizes->n_valid = excl + tot;
            sizes->n_bad = bad;
            sizes->f_opt = mn;
            sizes->n_plateau = 0;   // counted by the degree pass
        }
    }
    int32_t r[kSingleItems];
    int32_t id = local;
#pragma unroll
    for (int j = 0; j < kSingleItems; ++j) {
        if (valid_fitness(f[j])) {
            r[j] = excl + id;
            st_raw[id] = (int32_t)(base + j);
            st_fit[id] = f[j];
            ++id;
        } else {
            r[j] = -1;
        }
    }
    if (base + kSingleItems <= n_raw) {
#pragma unroll
        for (int q = 0; q < kSingleItems / 4; ++q)
            *reinterpret_cast<int4 *>(remap + base + 4 * q) = make_int4(r[4 * q], r[4 * q + 1], r[4 * q + 2], r[4 * q + 3]);
    } else {
#pragma unroll
        for (int j = 0; j < kSingleItems; ++j)
            if (base + j < n_raw) remap[base + j] = r[j];
    }
    __syncthreads();
    for (int32_t q = threadIdx.x; q < tot; q += kBlock) {
        valid_raw[excl + q] = st_raw[q];
        fit_c[excl + q] = st_fit[q];
    }
}

// ---------------------------------------------------------------------------
// FFG degrees (Sec. VII-B): for node v with raw index i and digits x, the
// candidate neighbours are c = i + (a - x_k) * stride_k (eq. 2: one parameter
// changed; adjacent: a = x_k +- 1 inside the list).  in_deg counts valid
// neighbours with strictly higher fitness (edges into v), out_deg those with
// strictly lower fitness (edges out of v).  The slot kernel also records the
// in-edges as a bit mask over the node's candidate slots.

// Bits [lo, hi) of a 64-bit word, 0 <= lo, hi <= 64.
__device__ __forceinline__ uint64_t range_bits(int32_t lo, int32_t hi) {
    return hi > lo ? ((~0ull >> (64 - hi)) & (~0ull << lo)) : 0ull;
}

// Set bits [lo, hi) of a W-word mask; the range lies inside slot run
// [run_lo, run_hi), whose words (uniform) bound the words touched.
template <int W>
__device__ __forceinline__ void set_bits(uint64_t (&m)[W], int32_t lo, int32_t hi, int32_t run_lo, int32_t run_hi) {
    const int32_t w0 = run_lo >> 6, w1 = (run_hi - 1) >> 6;
#pragma unroll
    for (int q = 0; q < W; ++q)
        if (q >= w0 && q <= w1)
            m[q] |= range_bits(min(max(lo - 64 * q, 0), 64), min(max(hi - 64 * q, 0), 64));
}

// Slot version.  A node's existing slots for parameter k are the last
// min(x_k, len) of the parameter's negative run and the first
// min(r_k - 1 - x_k, len) of its positive run, so the existence mask takes a
// few shifts per parameter.  The fitness gathers then run like the sweep's:
// a slot no lane of the wave has is skipped with a scalar branch, and lanes
// without it get the out-of-range buffer offset (the load returns 0, which
// no comparison below counts).
// SP and SL are SpaceDesc and SlotTable, either kernel arguments or entries
// of a segment table in the constant address space (scalar loads either way).
template <int W, bool BUF, class SP, class SL>
__device__ __forceinline__ void degree_slots(const SP &sp, const SL &sl, int32_t tile,
                                             const float *__restrict__ fit, int32_t fit_bytes,
                                             const int32_t *__restrict__ valid_raw, int32_t n,
                                             int32_t *__restrict__ in_deg, int32_t *__restrict__ out_deg,
                                             uint64_t *__restrict__ rec, uint64_t *__restrict__ presence,
                                             int32_t *__restrict__ off_table, int32_t k_pad,
                                             int64_t *__restrict__ tile_e, int32_t *__restrict__ tile_m,
                                             BuildSizes *__restrict__ sizes) {
    if (tile == 0) {
        // the sweep's offset table: raw offsets, then byte offsets from the
        // most negative (meaningful where the buffer-load sweep runs), 0 past k
        for (int32_t j = threadIdx.x; j < k_pad; j += kBlock) {
            const bool real = j < sl.k;
            off_table[j] = real ? sl.off[j] : 0;
            off_table[k_pad + j] = real ? (int32_t)(4u * ((uint32_t)sl.off[j] - (uint32_t)sl.off[0])) : 0;
        }
    }
    const int32_t v = tile * kBlock + threadIdx.x;
    const bool active = v < n;
    const uint32_t i = active ? (uint32_t)valid_raw[v] : 0u;
    const float fv = active ? fit[i] : 0.0f;
    uint64_t ex[W], m[W];
#pragma unroll
    for (int q = 0; q < W; ++q) ex[q] = m[q] = 0ull;
    if (active) {
        uint32_t qv = i;
        for (int k = sp.n - 1; k >= 0; --k) {   // digits, least significant first
            const uint32_t qn = (uint32_t)(((uint64_t)qv * sp.magic[k]) >> sp.shift[k]);
            const int32_t x = (int32_t)(qv - qn * (uint32_t)sp.radix[k]);
            qv = qn;
            const int32_t len = sl.blk_len[k];
            if (len <= 0) continue;
            const int32_t nb = sl.blk_neg[k], pb = sl.blk_pos[k];
            const int32_t a = min(x, len), bcnt = min(sp.radix[k] - 1 - x, len);
            set_bits<W>(ex, nb + len - a, nb + len, nb, nb + len);
            set_bits<W>(ex, pb, pb + bcnt, pb, pb + len);
        }
    }
    const __amdgpu_buffer_rsrc_t fr = __builtin_amdgcn_make_buffer_rsrc((void *)fit, (short)0, fit_bytes, 0x00020000);
    const uint32_t i4 = 4u * i;
    int32_t dout = 0;
    bool tie = false;
    // The comparisons work on the bits: by the time this pass runs every
    // fitness is positive and finite, +inf or NaN (the build stops on any
    // other), and positive finite floats order as their bit patterns, below
    // +inf (0x7f800000) and the NaNs.  A neighbour c is worse (an in-edge)
    // iff fv < c < +inf, i.e. (c - fv - 1) < (+inf - fv - 1) unsigned; better
    // (an out-edge) iff 0 < c < fv, i.e. (c - 1) < (fv - 1) unsigned, which
    // also drops the 0 of an absent slot.  Two VALU per test instead of two
    // float compares and an AND.
    const uint32_t fvb = __float_as_uint(fv);
    const uint32_t in_lo = fvb + 1u, in_span = 0x7f800000u - in_lo, out_hi = fvb - 1u;
#pragma unroll
    for (int b = 0; b < 2 * W; ++b) {
        if (32 * b >= sl.k) break;
        const uint32_t exb = (b & 1) ? (uint32_t)(ex[b >> 1] >> 32) : (uint32_t)ex[b >> 1];
        const uint32_t any = __builtin_amdgcn_readfirstlane(wave_or(exb));
        const uint32_t nex = ~exb;
        float fc[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            fc[u] = 0.0f;
            if ((any >> u) & 1u) {
                if (BUF) {
                    const uint32_t byte = ((nex << (31 - u)) & 0x80000000u) | (i4 + 4u * (uint32_t)sl.off[32 * b + u]);
                    fc[u] = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(fr, byte, 0, 0));
                } else {
                    fc[u] = ((exb >> u) & 1u) ? fit[(int32_t)i + sl.off[32 * b + u]] : 0.0f;
                }
            }
        }
        uint32_t inb = 0u;
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            // a neighbour that is worse (in-edge; +inf and NaN mark excluded
            // ones), or better (out-edge; 0 marks a slot the node does not have)
            if (W == 1) {
                // the same tests on floats: with one record word the compiler
                // turns the integer form into a 256-register kernel that spills
                if ((fc[u] > fv) & (fc[u] < INFINITY)) inb |= 1u << u;
                dout += (fc[u] < fv) & (fc[u] > 0.0f);
                tie |= fc[u] == fv;
            } else {
                const uint32_t cb = __float_as_uint(fc[u]);
                if (cb - in_lo < in_span) inb |= 1u << u;
                dout += cb - 1u < out_hi;
                tie |= cb == fvb;   // a valid neighbour of equal fitness (0, NaN, inf never equal fv)
            }
        }
        m[b >> 1] |= (b & 1) ? ((uint64_t)inb << 32) : (uint64_t)inb;
    }
    int32_t din = 0;
#pragma unroll
    for (int q = 0; q < W; ++q) din += __popcll(m[q]);
    if (active) {
        in_deg[v] = din;
        out_deg[v] = dout;
        const uint64_t tail = ((uint64_t)i << 32) | ((uint64_t)(uint32_t)dout << 24);
        uint64_t *p = rec + (int64_t)v * W;
#pragma unroll
        for (int q = 0; q < W; ++q) p[q] = m[q] | (q == W - 1 ? tail : 0ull);
    }
    // slots any node of this wave has as an in-edge (read by the sweep's scalar unit)
#pragma unroll
    for (int q = 0; q < W; ++q) {
        uint32_t lo = (uint32_t)m[q], hi = (uint32_t)(m[q] >> 32);
        lo = wave_or(lo);
        hi = wave_or(hi);
        if ((threadIdx.x & 63) == 0 && v < n) presence[(int64_t)(v >> 6) * W + q] = ((uint64_t)hi << 32) | lo;
    }
    const int64_t te = block_sum((int64_t)din);
    const int32_t tm = block_sum((int32_t)(v < n && dout == 0));
    const int32_t tp = block_sum((int32_t)(v < n && dout == 0 && tie));
    if (threadIdx.x == 0) {
        tile_e[tile] = te;
        tile_m[tile] = tm;
        if (tp > 0) atomicAdd(&sizes->n_plateau, tp);
    }
}

// One space: the descriptor is the kernel's only argument, read in place in
// the kernel-argument segment (a by-value table passed on by reference would
// otherwise be copied to private memory).
template <int W, bool BUF>
__global__ __launch_bounds__(kBlock) void k_degree_slots([[maybe_unused]] SegBuild arg) {
    const_ptr<SegBuild> g = kernel_arg<SegBuild>();
    degree_slots<W, BUF>(g->sp, g->sl, blockIdx.x, g->fit, g->fit_bytes, g->valid_raw, g->n, g->in_deg,
                         g->out_deg, g->rec, g->presence, g->off_table, g->k_pad, g->tile_e, g->tile_m, g->sizes);
}

// Generic count for spaces with more than kMaxSlots candidate slots: walks the
// parameters and their values directly.
template <bool ADJ>
__global__ __launch_bounds__(kBlock) void k_degree_generic(SpaceDesc sp, const float *__restrict__ fit,
                                                           const int32_t *__restrict__ valid_raw, int32_t n,
                                                           int32_t *__restrict__ in_deg,
                                                           int32_t *__restrict__ out_deg,
                                                           int64_t *__restrict__ tile_e,
                                                           int32_t *__restrict__ tile_m,
                                                           BuildSizes *__restrict__ sizes) {
    const int32_t v = blockIdx.x * kBlock + threadIdx.x;
    int32_t din = 0, dout = 0;
    bool tie = false;
    if (v < n) {
        const uint32_t i = (uint32_t)valid_raw[v];
        const float fv = fit[i];
        for (int k = 0; k < sp.n; ++k) {
            const uint32_t r = (uint32_t)sp.radix[k], st = (uint32_t)sp.stride[k];
            const uint32_t xk = (i / st) % r;
            const uint32_t row = i - xk * st;
            if (ADJ) {
                const float lo = xk > 0 ? fit[row + (xk - 1) * st] : NAN;
                const float hi = xk + 1 < r ? fit[row + (xk + 1) * st] : NAN;
                din += ((lo > fv) & (lo < INFINITY)) + ((hi > fv) & (hi < INFINITY));
                dout += (lo < fv) + (hi < fv);
                tie |= (lo == fv) | (hi == fv);
            } else {
                for (uint32_t a0 = 0; a0 < r; a0 += 8) {
                    float fc[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const uint32_t a = a0 + u;
                        fc[u] = (a < r && a != xk) ? fit[row + a * st] : NAN;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        din += (fc[u] > fv) & (fc[u] < INFINITY);
                        dout += (fc[u] < fv);
                        tie |= fc[u] == fv;
                    }
                }
            }
        }
        in_deg[v] = din;
        out_deg[v] = dout;
    }
    const int64_t te = block_sum((int64_t)din);
    const int32_t tm = block_sum((int32_t)(v < n && dout == 0));
    const int32_t tp = block_sum((int32_t)(v < n && dout == 0 && tie));
    if (threadIdx.x == 0) {
        tile_e[blockIdx.x] = te;
        tile_m[blockIdx.x] = tm;
        if (tp > 0) atomicAdd(&sizes->n_plateau, tp);
    }
}

__device__ __forceinline__ void degree_scan(const int64_t *__restrict__ tile_e, const int32_t *__restrict__ tile_m,
                                            int32_t n_tiles, int64_t *__restrict__ tile_eoff,
                                            int32_t *__restrict__ tile_moff, BuildSizes *__restrict__ sizes) {
    const int64_t e = scan_tiles(tile_e, tile_eoff, n_tiles);
    const int32_t m = scan_tiles(tile_m, tile_moff, n_tiles);
    if (threadIdx.x == 0) {
        sizes->n_edges = e;
        sizes->n_minima = m;
    }
}

// Exclusive prefix sum of one value per thread over a workgroup of B
// threads; *total receives the sum.
template <int B, typename T>
__device__ T block_excl_scan_b(T v, T *total) {
    __shared__ T part[B / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    T incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const T y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) part[wid] = incl;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < B / 64; ++w) {
        const T s = part[w];
        off += (w < wid) ? s : T(0);
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

// The degree pass's tile scans (edges and sinks) in one 1024-thread
// workgroup: each thread takes kScanItems consecutive tiles of both arrays,
// so up to 8192 tiles (2 M nodes) need one round of loads; larger spaces loop
// with a carry.  (The two-array, 256-thread scan_tiles took 14 us at the large
// workload, six dependent rounds.)
constexpr int kScanItems = 8;
__global__ __launch_bounds__(kFinishBlock) void k_degree_scan(const int64_t *__restrict__ tile_e,
                                                              const int32_t *__restrict__ tile_m,
                                                              int32_t n_tiles, int64_t *__restrict__ tile_eoff,
                                                              int32_t *__restrict__ tile_moff,
                                                              BuildSizes *__restrict__ sizes) {
    int64_t ce = 0;
    int32_t cm = 0;
    for (int32_t base = 0; base < n_tiles; base += kFinishBlock * kScanItems) {
        const int32_t first = base + (int32_t)threadIdx.x * kScanItems;
        int64_t e[kScanItems];
        int32_t m[kScanItems];
        int64_t se = 0;
        int32_t sm = 0;
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            const bool in = first + j < n_tiles;
            e[j] = in ? tile_e[first + j] : 0;
            m[j] = in ? tile_m[first + j] : 0;
            se += e[j];
            sm += m[j];
        }
        int64_t te;
        int32_t tm;
        int64_t re = ce + block_excl_scan_b<kFinishBlock>(se, &te);
        int32_t rm = cm + block_excl_scan_b<kFinishBlock>(sm, &tm);
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            if (first + j < n_tiles) {
                tile_eoff[first + j] = re;
                tile_moff[first + j] = rm;
            }
            re += e[j];
            rm += m[j];
        }
        ce += te;
        cm += tm;
    }
    if (threadIdx.x == 0) {
        sizes->n_edges = ce;
        sizes->n_minima = cm;
    }
}

// ---------------------------------------------------------------------------
// CSR fill: row_ptr by a workgroup scan of in_deg plus the tile offset, the
// minima (sinks) by a scan of the sink flags, then the sources of every
// in-edge in ascending raw (= node id) order.  Ascending order of
// c = i + (a - x_k) * stride_k is: below i, parameters 0..n-1 with a rising
// from 0 to x_k - 1; above i, parameters n-1..0 with a rising from x_k + 1.

// Shared prologue: row_ptr and minima for the workgroup's nodes.
__device__ __forceinline__ void fill_rows(int32_t tile, int32_t v, int32_t n, int32_t n_edges, int32_t din,
                                          int32_t sink, const int64_t *tile_eoff, const int32_t *tile_moff,
                                          int32_t *row_ptr, int32_t *minima, int32_t &e_off) {
    int32_t tot;
    e_off = (int32_t)tile_eoff[tile] + block_excl_scan(din, &tot);
    const int32_t m_off = tile_moff[tile] + block_excl_scan(sink, &tot);
    if (v < n) {
        row_ptr[v] = e_off;
        if (v == n - 1) row_ptr[n] = n_edges;
        if (sink) minima[m_off] = v;
    }
}

// Slot version: the in-edges come from the node records of the degree pass.
// Slots are sorted by raw-index offset, so a row's in-edges come out in
// ascending source id when every lane walks its set bits in slot order.  The
// remap gathers of a slot skip slots no lane of the wave needs (presence
// word) and use the out-of-range buffer offset for lanes whose bit is clear,
// as in the sweep.  The tile's rows are one contiguous range of col_idx; when
// it fits, it is assembled in LDS and written out with coalesced stores
// instead of one scattered 4-byte store per edge.
template <int W, bool BUF, class SL>
__device__ __forceinline__ void fill_slots(const SL &sl, int32_t tile, int32_t n_tiles,
                                           const int32_t *__restrict__ remap, int32_t remap_bytes,
                                           const uint64_t *__restrict__ rec, const uint64_t *__restrict__ presence,
                                           int32_t n, int32_t n_edges, const int32_t *__restrict__ in_deg,
                                           const int32_t *__restrict__ out_deg,
                                           const int64_t *__restrict__ tile_eoff,
                                           const int32_t *__restrict__ tile_moff, int32_t *__restrict__ row_ptr,
                                           int32_t *__restrict__ col_idx, int32_t *__restrict__ minima) {
    __shared__ int32_t stage[kFillStage];
    const int32_t v = tile * kBlock + threadIdx.x;
    const bool active = v < n;
    const int32_t din = active ? in_deg[v] : 0;
    const int32_t sink = (active && out_deg[v] == 0) ? 1 : 0;
    int32_t e_off;
    fill_rows(tile, v, n, n_edges, din, sink, tile_eoff, tile_moff, row_ptr, minima, e_off);
    const int64_t e_begin = tile_eoff[tile];
    const int64_t e_end = tile + 1 < n_tiles ? tile_eoff[tile + 1] : (int64_t)n_edges;
    const int32_t count = (int32_t)(e_end - e_begin);
    const bool staged = count <= kFillStage;   // uniform over the workgroup
    const __amdgpu_buffer_rsrc_t rr =
        __builtin_amdgcn_make_buffer_rsrc((void *)remap, (short)0, remap_bytes, 0x00020000);
    Record<W> r;
    if (active) {
        r = load_record<W>(rec, v);
    } else {
#pragma unroll
        for (int j = 0; j < W; ++j) r.w[j] = 0ull;
    }
    const int32_t i = r.raw();
    const uint32_t i4 = 4u * (uint32_t)i;
    const int32_t first = __builtin_amdgcn_readfirstlane(tile * kBlock + (int32_t)(threadIdx.x & ~63u));
    const_ptr<uint64_t> pw = to_const(presence) + (int64_t)(first >> 6) * W;
    const bool live = first < n;
    int32_t pos = e_off;
    const int32_t end = e_off + din;
#pragma unroll
    for (int b = 0; b < 2 * W; ++b) {
        if (32 * b >= sl.k || !live) break;
        const uint64_t pq = pw[b >> 1];
        const uint32_t any = (b & 1) ? (uint32_t)(pq >> 32) : (uint32_t)pq;
        const uint32_t bits = r.word32(b) & batch_mask(b, sl.k);
        const uint32_t nbits = ~bits;
        int32_t src[32];
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            src[u] = 0;
            if ((any >> u) & 1u) {
                if (BUF) {
                    const uint32_t byte = ((nbits << (31 - u)) & 0x80000000u) | (i4 + 4u * (uint32_t)sl.off[32 * b + u]);
                    src[u] = (int32_t)__builtin_amdgcn_raw_buffer_load_b32(rr, byte, 0, 0);
                } else {
                    src[u] = ((bits >> u) & 1u) ? remap[i + sl.off[32 * b + u]] : 0;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 32; ++u) {
            if (((bits >> u) & 1u) && pos < end) {
                if (staged)
                    stage[pos - (int32_t)e_begin] = src[u];
                else
                    col_idx[pos] = src[u];
                ++pos;
            }
        }
    }
    if (staged) {
        __syncthreads();
        for (int32_t j = threadIdx.x; j < count; j += kBlock) col_idx[e_begin + j] = stage[j];
    }
}

template <int W, bool BUF>
__global__ __launch_bounds__(kBlock) void k_fill_slots([[maybe_unused]] SegBuild arg) {
    const_ptr<SegBuild> g = kernel_arg<SegBuild>();
    fill_slots<W, BUF>(g->sl, blockIdx.x, gridDim.x, g->remap, g->remap_bytes, g->rec, g->presence, g->n,
                       g->n_edges, g->in_deg, g->out_deg, g->tile_eoff, g->tile_moff, g->row_ptr, g->col_idx,
                       g->minima);
}

// ---------------------------------------------------------------------------
// Segmented build: the same stages for every space of a batch in one launch.

__global__ __launch_bounds__(kBlock) void k_seg_compact_count(const SegBuild *__restrict__ segs,
                                                              const SegTile *__restrict__ tiles) {
    const_ptr<SegTile> t = to_const(tiles) + blockIdx.x;
    const_ptr<SegBuild> g = to_const(segs) + t->seg;
    compact_count(g->fit, g->sp.n_raw, t->tile, g->tile_cnt, g->tile_min, g->tile_bad);
}

__global__ __launch_bounds__(kBlock) void k_seg_compact_scan(const SegBuild *__restrict__ segs,
                                                             const int32_t *__restrict__ ids) {
    const_ptr<SegBuild> g = to_const(segs) + to_const(ids)[blockIdx.x];
    compact_scan(g->tile_cnt, g->tile_min, g->tile_bad, g->c_tiles, g->tile_off, g->sizes);
}

__global__ __launch_bounds__(kBlock) void k_seg_compact_write(const SegBuild *__restrict__ segs,
                                                              const SegTile *__restrict__ tiles) {
    const_ptr<SegTile> t = to_const(tiles) + blockIdx.x;
    const_ptr<SegBuild> g = to_const(segs) + t->seg;
    compact_write(g->fit, g->sp.n_raw, t->tile, g->tile_off, g->remap, g->valid_raw, g->fit_c);
}

template <int W, bool BUF>
__global__ __launch_bounds__(kBlock) void k_seg_degree(const SegBuild *__restrict__ segs,
                                                       const SegTile *__restrict__ tiles) {
    const_ptr<SegTile> t = to_const(tiles) + blockIdx.x;
    const_ptr<SegBuild> g = to_const(segs) + t->seg;
    degree_slots<W, BUF>(g->sp, g->sl, t->tile, g->fit, g->fit_bytes, g->valid_raw, g->n, g->in_deg, g->out_deg,
                         g->rec, g->presence, g->off_table, g->k_pad, g->tile_e, g->tile_m, g->sizes);
}

__global__ __launch_bounds__(kBlock) void k_seg_degree_scan(const SegBuild *__restrict__ segs,
                                                            const int32_t *__restrict__ ids) {
    const_ptr<SegBuild> g = to_const(segs) + to_const(ids)[blockIdx.x];
    degree_scan(g->tile_e, g->tile_m, g->n_tiles, g->tile_eoff, g->tile_moff, g->sizes);
}

template <int W, bool BUF>
__global__ __launch_bounds__(kBlock) void k_seg_fill(const SegBuild *__restrict__ segs,
                                                     const SegTile *__restrict__ tiles) {
    const_ptr<SegTile> t = to_const(tiles) + blockIdx.x;
    const_ptr<SegBuild> g = to_const(segs) + t->seg;
    fill_slots<W, BUF>(g->sl, t->tile, g->n_tiles, g->remap, g->remap_bytes, g->rec, g->presence, g->n,
                       g->n_edges, g->in_deg, g->out_deg, g->tile_eoff, g->tile_moff, g->row_ptr, g->col_idx,
                       g->minima);
}

// Generic version for spaces with more than kMaxSlots candidate slots.
template <bool ADJ>
__global__ __launch_bounds__(kBlock) void k_fill_generic(SpaceDesc sp, const float *__restrict__ fit,
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
    int32_t e_off;
    fill_rows(blockIdx.x, v, n, n_edges, din, sink, tile_eoff, tile_moff, row_ptr, minima, e_off);
    if (v >= n || din == 0) return;
    const uint32_t i = (uint32_t)valid_raw[v];
    const float fv = fit[i];
    const int32_t end = e_off + din;
    int32_t pos = e_off;
    auto take = [&](uint32_t c) {
        const float fc = fit[c];
        if ((fc > fv) & (fc < INFINITY)) {
            if (pos < end) col_idx[pos] = remap[c];
            ++pos;
        }
    };
    for (int k = 0; k < sp.n; ++k) {  // below i
        const uint32_t r = (uint32_t)sp.radix[k], st = (uint32_t)sp.stride[k];
        const uint32_t xk = (i / st) % r;
        const uint32_t row = i - xk * st;
        if (ADJ) {
            if (xk > 0) take(row + (xk - 1) * st);
        } else {
            for (uint32_t a = 0; a < xk; ++a) take(row + a * st);
        }
    }
    for (int k = sp.n - 1; k >= 0; --k) {  // above i
        const uint32_t r = (uint32_t)sp.radix[k], st = (uint32_t)sp.stride[k];
        const uint32_t xk = (i / st) % r;
        const uint32_t row = i - xk * st;
        if (ADJ) {
            if (xk + 1 < r) take(row + (xk + 1) * st);
        } else {
            for (uint32_t a = xk + 1; a < r; ++a) take(row + a * st);
        }
    }
}

// ---------------------------------------------------------------------------
// PageRank power iteration (Sec. VII-B) with damping d, uniform teleport and
// sink mass spread uniformly:
//   r'[w] = d * sum_{u->w} r[u]/out_deg(u) + (d * sum_{sinks} r + 1 - d) / N.
// Stored iterate y_k = r_k up to s_k = 1/sum(y_k); x_k = y_k/out_deg.  The
// edge sum is FP32; the per-node affine update, the residual
// ||r_{k+1} - r_k||_1, the renormalisation and the sink mass are FP64.
//
// Each tile of kBlock nodes (each workgroup for the CSR sweep) writes its
// three FP64 sums (sum y', sum |y' - r|, sum of y' over sinks) to its slot of
// a partials array; a one-workgroup kernel then reduces them in a fixed order
// and sets s, c, the residual and the stop flag for the next sweep.  (Having
// the last workgroup of the sweep do this instead needs an agent-scope
// release from every workgroup, which costs more than the extra launch.)

// Sum three values over the workgroup (valid in every thread), fixed tree.
template <int B = kBlock>
__device__ void block_sum3(double &a, double &b, double &c) {
    __shared__ double part[3][B / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    if (lane == 0) {
        part[0][wid] = a;
        part[1][wid] = b;
        part[2][wid] = c;
    }
    __syncthreads();
    a = part[0][0];
    b = part[1][0];
    c = part[2][0];
#pragma unroll
    for (int w = 1; w < B / 64; ++w) {
        a += part[0][w];
        b += part[1][w];
        c += part[2][w];
    }
    __syncthreads();
}

__device__ __forceinline__ void write_partials(double *partials, int32_t j, double ps, double pr, double pk) {
    block_sum3(ps, pr, pk);
    if (threadIdx.x == 0) {
        double *pp = partials + 3 * (int64_t)j;
        pp[0] = ps;
        pp[1] = pr;
        pp[2] = pk;
    }
}

// Reduce `count` partial triples in a fixed order and set up the next step.
// One workgroup of kFinishBlock threads.  The triples are read as one flat
// array with consecutive threads on consecutive doubles; rounds of
// 3 kFinishBlock elements keep the component of a thread's q-th element of
// a round fixed at (threadIdx.x + q kFinishBlock) mod 3.  first: the triples
// come from the initial iterate.
__device__ void finish_step(PrState *st, const double *__restrict__ partials, int32_t count, double d, double tol,
                            int32_t max_iter, int32_t n, bool first, bool exact = false) {
    constexpr int B = kFinishBlock, kRound = 3 * B;
    const int64_t total = 3 * (int64_t)count;
    double r[3] = {0.0, 0.0, 0.0};   // r[q]: component (threadIdx.x + q B) mod 3
    // 24 loads in flight per thread: one round covers 8192 tiles (2 M nodes)
    constexpr int kU = 8;
    for (int64_t e0 = 0; e0 < total; e0 += kU * kRound) {
        double v[kU][3];
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int64_t e = e0 + u * kRound + q * B + threadIdx.x;
                v[u][q] = e < total ? partials[e] : 0.0;
            }
#pragma unroll
        for (int u = 0; u < kU; ++u)
#pragma unroll
            for (int q = 0; q < 3; ++q) r[q] += v[u][q];
    }
    static_assert(B % 3 == 1, "component rotation assumes B = 1 mod 3");
    const int c0 = threadIdx.x % 3;   // component of r[0]; r[q] holds component (c0 + q) mod 3
    double s0 = c0 == 0 ? r[0] : (c0 == 2 ? r[1] : r[2]);
    double s1 = c0 == 1 ? r[0] : (c0 == 0 ? r[1] : r[2]);
    double s2 = c0 == 2 ? r[0] : (c0 == 1 ? r[1] : r[2]);
    block_sum3<B>(s0, s1, s2);
    if (first && threadIdx.x == 0) {
        // lagged step: r_0 = w_0 (no constant term), so sweep 0 adds nothing
        // and sweep 1 adds gamma_0 = (d sink(r_0) + 1 - d) / N
        st->gam[0][0] = st->gam[0][1] = 0.0;
        st->gam[1][0] = exact ? 0.0 : (d * s2 + (1.0 - d)) / (double)n;
        st->gam[1][1] = 0.0;
        st->out_buf = 0;
        st->out_gamma = 0.0;
        st->out_sigma = s0;
    }
    if (exact && threadIdx.x == 0) {
        // Jacobi sweeps y' = d P y + 1 (the sweep computes s d acc + c with
        // s = c = 1); a sweep that changes no value ends them, and s then
        // scales the fixed point to sum 1 for the output
        st->sigma = s0;
        st->sink = s2;
        st->c = 1.0;
        if (first) {
            st->s = 1.0;
            st->k = 0;
            st->done = 0;
            st->worked = 0;
            st->resid = 0.0;
            st->resid_prev = 0.0;
        } else {
            st->resid_prev = st->resid;
            st->resid = s1;
            st->k += 1;
            st->worked += 1;
            st->s = 1.0;
            if (s1 == 0.0)
                st->done = 1;
            else if (st->k >= max_iter)
                st->done = 2;
            if (st->done) st->s = 1.0 / s0;
        }
        return;
    }
    if (threadIdx.x == 0) {
        const double s = 1.0 / s0;
        st->sigma = s0;
        st->sink = s2;
        st->s = s;
        st->c = (d * s2 * s + (1.0 - d)) / (double)n;
        if (first) {
            st->k = 0;
            st->done = 0;
            st->worked = 0;
            st->resid = 0.0;
            st->resid_prev = 0.0;
        } else {
            st->resid_prev = st->resid;
            st->resid = s1;
            st->k += 1;
            st->worked += 1;
            if (s1 < tol)
                st->done = 1;
            else if (st->k >= max_iter)
                st->done = 2;
        }
    }
}

// Step kernel: skipped, like the sweep it follows, once the stop flag is set.
template <bool FIRST>
__global__ __launch_bounds__(kFinishBlock) void k_pr_finish(PrArgs a, int32_t count) {
    if (!FIRST && a.st->done) return;
    finish_step(a.st, a.partials, count, a.d, a.tol, a.max_iter, a.n, FIRST, a.exact != 0);
}

// ---------------------------------------------------------------------------
// Lagged step.  With the plain power iteration, the step kernel between two
// sweeps costs about a fifth of an iteration at the large workload, mostly
// the fixed cost of a launch.  In the lagged form every sweep runs straight
// after the previous one, and its workgroup 0 first does the step of the
// sweep before.  A sweep therefore cannot know the constant term of its own
// input r_j = w_j + gamma_{j-1}, gamma = (d sink(r) + 1 - d) / N being a
// reduction over that input, nor the residual of r_j, which needs
// gamma_{j-1} as well.  It stores w_{j+1} = d (P^T D^-1 w_j + gamma_{j-1}
// P^T D^-1 1) without its constant, P^T D^-1 1 coming from the first
// sweep's edge sums (PrArgs::g), and adds the residual of r_j against
// r_{j-1} from the stored w_j and w_{j-1}.  The iterates are those of the
// plain iteration in exact arithmetic; the stop is seen one sweep later.

// The stop flag of the lagged step.  Workgroup 0 sets it while the rest of
// its sweep still runs; the other waves read it at device scope ahead of
// each tile and stop sweeping once it is set (their results are not used
// any more), so the sweep after the stop costs little more than its first
// tiles.
__device__ __forceinline__ void set_stop(PrState *st, int32_t v) {
    __hip_atomic_store(&st->done, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t peek_stop(const PrState *st) {
    return __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(const_cast<int32_t *>(&st->done), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Workgroup 0 of sweep j >= 1: reduce the partial triples of sweep j - 1
// in a fixed order (thread t sums parts t, t + kBlock, ...; then a fixed
// tree) and do its step.  Sweep j - 1 wrote sum w_j, the residual
// |r_{j-1} - r_{j-2}| (zero for j = 1) and the sink part of sum w_j; for
// the exact method, sum y_j, |y_j - y_{j-1}| and the sink part.
__device__ void lag_step(const PrArgs &a) {
    const int32_t j = a.sweep;
    const int64_t stride = a.part_stride;
    const double *__restrict__ p = a.partials + (int64_t)((j - 1) & 1) * 3 * stride;
    constexpr int kU = 8;   // 24 loads in flight: one round covers 2048 workgroups
    double r0 = 0.0, r1 = 0.0, r2 = 0.0;
    for (int32_t i0 = 0; i0 < a.n_parts; i0 += kU * kBlock) {
        double v[3][kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int32_t i = i0 + u * kBlock + (int32_t)threadIdx.x;
            const bool ok = i < a.n_parts;
            v[0][u] = ok ? p[i] : 0.0;
            v[1][u] = ok ? p[stride + i] : 0.0;
            v[2][u] = ok ? p[2 * stride + i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            r0 += v[0][u];
            r1 += v[1][u];
            r2 += v[2][u];
        }
    }
    block_sum3(r0, r1, r2);
    if (threadIdx.x != 0) return;
    PrState *st = a.st;
    if (a.exact) {
        // y_j is final once a sweep changed nothing
        st->resid_prev = st->resid;
        st->resid = r1;
        st->k = j;
        st->worked = j;
        st->sigma = r0;
        st->sink = r2;
        const int32_t stop = r1 == 0.0 ? 1 : (j >= a.max_iter ? 2 : 0);
        if (stop) {
            st->out_buf = j % 3;
            st->out_gamma = 0.0;
            st->out_sigma = r0;
            set_stop(st, stop);
        }
        return;
    }
    const double ga = st->gam[j & 1][0], gb = st->gam[j & 1][1];   // gamma_{j-1}, gamma_{j-2}
    const double n = (double)a.n;
    const double sig = r0 + n * ga;                        // sum of r_j
    const double sink = r2 + (double)a.n_sinks * ga;       // sink mass of r_j
    if (j >= 2) {
        st->resid_prev = st->resid;
        st->resid = r1;
        st->k = j - 1;
        st->worked = j - 1;
        const int32_t stop = r1 < a.tol ? 1 : (j - 1 >= a.max_iter ? 2 : 0);
        if (stop) {
            // r_{j-1} = w_{j-1} + gamma_{j-2}, summed by the previous step
            st->out_buf = (j - 1) % 3;
            st->out_gamma = gb;
            st->out_sigma = st->sigma;
            set_stop(st, stop);
        }
    }
    st->gam[(j + 1) & 1][0] = (a.d * sink + (1.0 - a.d)) / n;   // gamma_j
    st->gam[(j + 1) & 1][1] = ga;
    st->sigma = sig;
    st->sink = sink;
}

// One partial triple per workgroup (lagged step), to buffer sweep & 1.
__device__ __forceinline__ void write_lag_partials(const PrArgs &a, double ps, double pr, double pk) {
    block_sum3(ps, pr, pk);
    if (threadIdx.x == 0) {
        const int64_t stride = a.part_stride;
        double *pp = a.partials + (int64_t)(a.sweep & 1) * 3 * stride + blockIdx.x;
        pp[0] = ps;
        pp[stride] = pr;
        pp[2 * stride] = pk;
    }
}

// What a lagged sweep needs besides its iterate: the constant terms
// gamma_{j-1} (ga) and gamma_{j-2} (gb), ga / y0 (gs), and the mode.
enum LagMode : int32_t { kLagFirst = 0, kLagNext = 1, kLagExact = 2 };
struct LagTerms {
    const float *y_prev;   // w_{j-1}
    float *g;              // P^T D^-1 1 times y0 (written by the first sweep)
    double ga, gb, gs, d;
    int32_t mode;
};

__device__ __forceinline__ LagTerms lag_terms(const PrArgs &a) {
    LagTerms t;
    const int32_t j = a.sweep;
    t.y_prev = a.y[(j + 2) % 3];
    t.g = a.g;
    t.d = a.d;
    t.mode = a.exact ? kLagExact : (j == 0 ? kLagFirst : kLagNext);
    const PrState *st = a.st;
    t.ga = st->gam[j & 1][0];
    t.gb = st->gam[j & 1][1];
    const double y0 = (double)(float)(1.0 / (double)a.n);
    t.gs = t.ga / y0;
    return t;
}

// Whether a lagged sweep has node work: the sweep after the last iteration
// the cap allows only does the step of the one before.
__device__ __forceinline__ bool lag_has_tiles(const PrArgs &a) {
    return a.sweep <= a.max_iter - (a.exact ? 1 : 0);
}

// The new value of node v in a lagged sweep from its edge sum acc, its terms
// of the three partial sums, and (first sweep) its entry of g.  yin = w_j[v],
// yprev = w_{j-1}[v] and gv = g[v] are loaded by the caller in every mode
// (uninitialised in the modes that do not use them: not read here).
__device__ __forceinline__ float lag_node(const LagTerms &t, int32_t v, float acc, float yin, float yprev, float gv,
                                          int32_t deg, double &ps, double &pr, double &pk) {
    double w;
    if (t.mode == kLagExact)
        w = t.d * (double)acc + 1.0;
    else if (t.mode == kLagFirst)
        w = t.d * (double)acc;
    else
        w = t.d * ((double)acc + t.gs * (double)gv);
    const float yf = (float)w;
    ps += (double)yf;
    if (t.mode == kLagExact)
        pr += fabs((double)yf - (double)yin);
    else if (t.mode == kLagNext)
        pr += fabs(((double)yin + t.ga) - ((double)yprev + t.gb));
    else
        t.g[v] = acc;
    if (deg == 0) pk += (double)yf;
    return yf;
}

// Initial iterate r = 1/N of one tile of kBlock nodes, with its partial sums.
__device__ __forceinline__ void init_tile(int32_t tile, int32_t n, const int32_t *__restrict__ out_deg,
                                          const int32_t *__restrict__ xmap, float *y0v, float *x0v,
                                          double *partials) {
    const int32_t v = tile * kBlock + threadIdx.x;
    const float y0 = (float)(1.0 / (double)n);
    double ps = 0.0, pk = 0.0;
    if (v < n) {
        const int32_t deg = out_deg[v];
        y0v[v] = y0;
        x0v[xmap ? xmap[v] : v] = deg > 0 ? y0 / (float)deg : 0.0f;
        ps = (double)y0;
        if (deg == 0) pk = (double)y0;
    }
    write_partials(partials, tile, ps, 0.0, pk);
}

__global__ __launch_bounds__(kBlock) void k_pr_init(PrArgs a) {
    const int32_t n_tiles = (a.n + kBlock - 1) / kBlock;
    for (int32_t t = blockIdx.x; t < n_tiles; t += gridDim.x)
        init_tile(t, a.n, a.out_deg, a.kind == kSweepSlots ? a.valid_raw : nullptr, a.y[0], a.x[0], a.partials);
}

// Lagged step: the initial iterate without partial sums and without a step
// kernel.  Its sums are known: N y0 and M y0 over the M sinks, exact in FP64
// (y0 = 1/N in FP32 has 24 significant bits), as the reduction of the
// plain path gives them; workgroup 0 writes the state of the first step.
__global__ __launch_bounds__(kBlock) void k_pr_init_lag(PrArgs a) {
    const float y0 = (float)(1.0 / (double)a.n);
    const int32_t *xmap = a.kind == kSweepSlots ? a.valid_raw : nullptr;
    for (int32_t v = blockIdx.x * kBlock + threadIdx.x; v < a.n; v += gridDim.x * kBlock) {
        const int32_t deg = a.out_deg[v];
        a.y[0][v] = y0;
        a.x[0][xmap ? xmap[v] : v] = deg > 0 ? y0 / (float)deg : 0.0f;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        PrState *st = a.st;
        const double y = (double)y0, n = (double)a.n;
        const double s0 = n * y, s2 = (double)a.n_sinks * y;
        st->sigma = s0;
        st->sink = s2;
        st->s = a.exact ? 1.0 : 1.0 / s0;
        st->c = a.exact ? 1.0 : (a.d * s2 * st->s + (1.0 - a.d)) / n;
        st->k = 0;
        st->done = 0;
        st->worked = 0;
        st->resid = 0.0;
        st->resid_prev = 0.0;
        // sweep 0 adds nothing (r_0 = w_0), sweep 1 adds gamma_0
        st->gam[0][0] = st->gam[0][1] = 0.0;
        st->gam[1][0] = a.exact ? 0.0 : (a.d * s2 + (1.0 - a.d)) / n;
        st->gam[1][1] = 0.0;
        st->out_buf = 0;
        st->out_gamma = 0.0;
        st->out_sigma = s0;
    }
}

// Tiles of the persistent grid.  XCD j = b % 8 owns the contiguous j-th
// eighth of the tiles, and its workgroups take consecutive tiles in turn, so
// at any time an XCD sweeps a narrow band of nodes and the x values that band
// gathers stay in its L2.
struct TileWalk {
    int32_t first, end, step;
    __device__ TileWalk(int32_t n_tiles) {
        const int g = gridDim.x;
        const int xcd = blockIdx.x % kXcds;
        const int32_t per = (n_tiles + kXcds - 1) / kXcds;
        const int32_t lo = per * xcd, hi = min(per * (xcd + 1), n_tiles);
        const int nb = g / kXcds, l = blockIdx.x / kXcds;
        first = lo + l;
        end = hi;
        step = nb;
    }
};

__device__ __forceinline__ void pr_node_update(const PrArgs &a, int32_t v, int32_t xi, float acc, double sd,
                                               double c, double s, const float *y_in, float *y_out,
                                               float *x_out, double &ps, double &pr, double &pk) {
    const float yf = (float)(sd * (double)acc + c);
    const int32_t deg = a.out_deg[v];
    y_out[v] = yf;
    x_out[xi] = deg > 0 ? yf / (float)deg : 0.0f;
    ps += (double)yf;
    pr += fabs((double)yf - s * (double)y_in[v]);
    if (deg == 0) pk += (double)yf;
}

// CSR sweep, L lanes per row: the lanes of a row read consecutive col_idx
// entries (four rounds of loads in flight) and reduce with shuffles.
// LAG: the lagged step (see lag_step).
template <int L, bool LAG>
__global__ __launch_bounds__(kBlock) void k_pr_iter_csr(PrArgs a) {
    const PrState *st = a.st;
    if (st->done) return;
    if (LAG) {
        if (blockIdx.x == 0 && a.sweep >= 1) lag_step(a);
        if (!lag_has_tiles(a)) return;
    }
    const int32_t k = LAG ? a.sweep : st->k;
    const float *__restrict__ y_in = a.y[LAG ? k % 3 : k & 1];
    const float *__restrict__ x_in = a.x[k & 1];
    float *__restrict__ y_out = a.y[LAG ? (k + 1) % 3 : (k + 1) & 1];
    float *__restrict__ x_out = a.x[(k + 1) & 1];
    LagTerms lt{};
    if (LAG) lt = lag_terms(a);
    const int32_t *__restrict__ row_ptr = a.row_ptr;
    const int32_t *__restrict__ col_idx = a.col_idx;
    const double s = LAG ? 1.0 : st->s, c = LAG ? 0.0 : st->c;
    const double sd = s * a.d;
    constexpr int kRows = kBlock / L;
    const int lane = threadIdx.x % L;
    const int sub = threadIdx.x / L;
    const TileWalk w((a.n + kRows - 1) / kRows);
    double ps = 0.0, pr = 0.0, pk = 0.0;
    for (int32_t t = w.first; t < w.end; t += w.step) {
        const int32_t stop = LAG ? peek_stop(a.st) : 0;
        const int32_t v = t * kRows + sub;
        float acc = 0.0f;
        // lagged step: the row's own values, loaded ahead of its gathers
        int32_t deg = 0;
        float yin = 0.0f, yprev = 0.0f, gv = 0.0f;
        if (LAG && lane == 0 && v < a.n) {
            deg = a.out_deg[v];
            yin = y_in[v];
            yprev = lt.y_prev[v];
            gv = lt.g[v];
        }
        if (v < a.n) {
            const int32_t e1 = row_ptr[v + 1];
            for (int32_t e = row_ptr[v] + lane; e < e1; e += 4 * L) {
                int32_t cix[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) cix[u] = e + u * L < e1 ? col_idx[e + u * L] : -1;
                float xv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) xv[u] = cix[u] >= 0 ? x_in[cix[u]] : 0.0f;
#pragma unroll
                for (int u = 0; u < 4; ++u) acc += xv[u];
            }
        }
#pragma unroll
        for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0 && v < a.n) {
            if (LAG) {
                const float yf = lag_node(lt, v, acc, yin, yprev, gv, deg, ps, pr, pk);
                y_out[v] = yf;
                x_out[v] = deg > 0 ? yf / (float)deg : 0.0f;
            } else {
                pr_node_update(a, v, v, acc, sd, c, s, y_in, y_out, x_out, ps, pr, pk);
            }
        }
        if (stop) break;   // lagged step, per wave: this loop has no barrier
    }
    if (LAG)
        write_lag_partials(a, ps, pr, pk);
    else
        write_partials(a.partials, blockIdx.x, ps, pr, pk);
}


// ---------------------------------------------------------------------------
// Rows binned by in-degree (BinTable): each class of buckets has its own lanes
// per row L and T blocks of kBlock / L rows per tile.  A row's terms are
// gathered through the CSR exactly as in k_pr_iter_csr<L> and reduced over
// its L lanes with shuffles; x is indexed by node id.

struct BinSweep {
    const int32_t *row_ptr, *col_idx, *out_deg, *rows;
    const float *y_in, *x_in;
    float *y_out, *x_out;
    double s, c, sd;
    LagTerms lt;   // lagged step only
};

template <int L, bool LAG>
__device__ __forceinline__ void binned_block(const BinSweep &q, int32_t first, int32_t count, double &ps,
                                             double &pr, double &pk) {
    const int lane = threadIdx.x % L;
    const int32_t r = first + (int32_t)(threadIdx.x / L);
    const bool live = r < count;
    const int32_t v = live ? q.rows[r] : 0;
    float acc = 0.0f;
    // lagged step: the row's own values, loaded ahead of its gathers
    int32_t ldeg = 0;
    float yin = 0.0f, yprev = 0.0f, gv = 0.0f;
    if (LAG && lane == 0 && live) {
        ldeg = q.out_deg[v];
        yin = q.y_in[v];
        yprev = q.lt.y_prev[v];
        gv = q.lt.g[v];
    }
    if (live) {
        const int32_t e1 = q.row_ptr[v + 1];
        for (int32_t e = q.row_ptr[v] + lane; e < e1; e += 4 * L) {
            int32_t cix[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) cix[u] = e + u * L < e1 ? q.col_idx[e + u * L] : -1;
            float xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] = cix[u] >= 0 ? q.x_in[cix[u]] : 0.0f;
#pragma unroll
            for (int u = 0; u < 4; ++u) acc += xv[u];
        }
    }
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0 && live) {
        if (LAG) {
            const float yf = lag_node(q.lt, v, acc, yin, yprev, gv, ldeg, ps, pr, pk);
            q.y_out[v] = yf;
            q.x_out[v] = ldeg > 0 ? yf / (float)ldeg : 0.0f;
        } else {
            const int32_t deg = q.out_deg[v];
            const float yf = (float)(q.sd * (double)acc + q.c);
            q.y_out[v] = yf;
            q.x_out[v] = deg > 0 ? yf / (float)deg : 0.0f;
            ps += (double)yf;
            pr += fabs((double)yf - q.s * (double)q.y_in[v]);
            if (deg == 0) pk += (double)yf;
        }
    }
}

// Tile t (0 <= t < table.tiles) of a binned sweep: its class, then T blocks,
// their terms added to ps, pr, pk.  The table is read in place (kernel
// arguments or the member table) through the scalar unit.
template <bool LAG>
__device__ __forceinline__ void binned_tile(const BinSweep &q0, const_ptr<BinTable> tb, int32_t t, double &ps,
                                            double &pr, double &pk) {
    int cl = 0;
    const int nc = tb->n_classes;
    for (int j = 1; j < nc; ++j)
        if (t >= tb->c[j].tile_begin) cl = j;
    const const_ptr<BinClass> c = &tb->c[cl];
    const int32_t rows = c->rows, lanes = c->lanes, blocks = c->blocks;
    BinSweep q = q0;
    q.rows = q0.rows + c->row_begin;
    const int32_t lt = t - c->tile_begin;
    for (int b = 0; b < blocks; ++b) {
        const int32_t first = (lt * blocks + b) * (kBlock / lanes);
        switch (lanes) {
            case 1: binned_block<1, LAG>(q, first, rows, ps, pr, pk); break;
            case 2: binned_block<2, LAG>(q, first, rows, ps, pr, pk); break;
            case 4: binned_block<4, LAG>(q, first, rows, ps, pr, pk); break;
            case 8: binned_block<8, LAG>(q, first, rows, ps, pr, pk); break;
            case 16: binned_block<16, LAG>(q, first, rows, ps, pr, pk); break;
            case 32: binned_block<32, LAG>(q, first, rows, ps, pr, pk); break;
            default: binned_block<64, LAG>(q, first, rows, ps, pr, pk); break;
        }
    }
}

// The binned sweep over the tiles of a.bins (the plan's whole table, or a
// part of it while the autotuner times one class).  LAG: the lagged step.
template <bool LAG>
__global__ __launch_bounds__(kBlock) void k_pr_iter_binned(PrArgs a) {
    const PrState *st = a.st;
    if (st->done) return;
    if (LAG) {
        if (blockIdx.x == 0 && a.sweep >= 1) lag_step(a);
        if (!lag_has_tiles(a)) return;
    }
    const int32_t k = LAG ? a.sweep : st->k;
    BinSweep q;
    q.row_ptr = a.row_ptr;
    q.col_idx = a.col_idx;
    q.out_deg = a.out_deg;
    q.rows = a.bin_rows;
    q.y_in = a.y[LAG ? k % 3 : k & 1];
    q.x_in = a.x[k & 1];
    q.y_out = a.y[LAG ? (k + 1) % 3 : (k + 1) & 1];
    q.x_out = a.x[(k + 1) & 1];
    if (LAG) {
        q.s = q.c = q.sd = 0.0;
        q.lt = lag_terms(a);
    } else {
        q.s = st->s;
        q.c = st->c;
        q.sd = q.s * a.d;
    }
    // Every class's tiles are dealt to the XCDs in eighths, XCD j taking the
    // j-th eighth of each class in turn: a class's rows ascend in node id,
    // so an XCD works in about the j-th eighth of the nodes whatever the
    // class, and the x values its rows gather stay local to its L2.
    const const_ptr<BinTable> tb = &kernel_arg<PrArgs>()->bins;
    const int xcd = blockIdx.x % kXcds, nb = gridDim.x / kXcds, l = blockIdx.x / kXcds;
    const int nc = tb->n_classes;
    double ws = 0.0, wr = 0.0, wk = 0.0;   // lagged step: the workgroup's sums
    bool stopped = false;                  // lagged step: the stop flag was seen (per wave)
    for (int cl = 0; cl < nc && !stopped; ++cl) {
        const int32_t t0 = tb->c[cl].tile_begin;
        const int32_t ct = (cl + 1 < nc ? tb->c[cl + 1].tile_begin : a.bins.tiles) - t0;
        const int32_t per = (ct + kXcds - 1) / kXcds;
        const int32_t lo = t0 + per * xcd, hi = t0 + min(per * (xcd + 1), ct);
        for (int32_t t = lo + l; t < hi; t += nb) {
            if (LAG) {
                const int32_t stop = peek_stop(a.st);
                binned_tile<true>(q, tb, t, ws, wr, wk);
                if (stop) {   // per wave: no barrier in the tile loop
                    stopped = true;
                    break;
                }
            } else {
                double ps = 0.0, pr = 0.0, pk = 0.0;
                binned_tile<false>(q, tb, t, ps, pr, pk);
                write_partials(a.partials, t, ps, pr, pk);
            }
        }
    }
    if (LAG) write_lag_partials(a, ws, wr, wk);
}

// Binning of the rows: per node tile, the number of rows of each class;
// one-workgroup scan of those counts in class-major order; then every row
// written to its class's range in ascending node id.
__device__ __forceinline__ int8_t row_class(const int32_t *__restrict__ row_ptr, int32_t v, int32_t n,
                                            const int8_t *__restrict__ class_of) {
    return v < n ? class_of[bucket_of(row_ptr[v + 1] - row_ptr[v])] : (int8_t)-1;
}

__global__ __launch_bounds__(kBlock) void k_bin_count(const int32_t *__restrict__ row_ptr, int32_t n,
                                                      const int8_t *__restrict__ class_of,
                                                      int32_t *__restrict__ cnt, int32_t n_tiles) {
    __shared__ int32_t wc[kBuckets][kBlock / 64];
    const int32_t tile = blockIdx.x, v = tile * kBlock + threadIdx.x;
    const int8_t cls = row_class(row_ptr, v, n, class_of);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < kBuckets; ++c) {
        const uint64_t m = __ballot(cls == c);
        if (lane == 0) wc[c][wid] = __popcll(m);
    }
    __syncthreads();
    if (threadIdx.x < kBuckets) {
        int32_t t = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) t += wc[threadIdx.x][w];
        cnt[(int64_t)threadIdx.x * n_tiles + tile] = t;
    }
}

__global__ __launch_bounds__(kBlock) void k_bin_scan(const int32_t *__restrict__ cnt, int32_t *__restrict__ off,
                                                     int32_t *__restrict__ totals, int32_t n_tiles) {
    const int32_t total = scan_tiles(cnt, off, kBuckets * n_tiles);
    __syncthreads();
    if (threadIdx.x < kBuckets) {
        const int c = threadIdx.x;
        const int32_t lo = off[(int64_t)c * n_tiles];
        const int32_t hi = c + 1 < kBuckets ? off[(int64_t)(c + 1) * n_tiles] : total;
        totals[c] = hi - lo;
    }
}

__global__ __launch_bounds__(kBlock) void k_bin_write(const int32_t *__restrict__ row_ptr, int32_t n,
                                                      const int8_t *__restrict__ class_of,
                                                      const int32_t *__restrict__ off, int32_t n_tiles,
                                                      int32_t *__restrict__ bin_rows) {
    __shared__ int32_t wc[kBuckets][kBlock / 64];
    const int32_t tile = blockIdx.x, v = tile * kBlock + threadIdx.x;
    const int8_t cls = row_class(row_ptr, v, n, class_of);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int32_t rank = 0;
#pragma unroll
    for (int c = 0; c < kBuckets; ++c) {
        const uint64_t m = __ballot(cls == c);
        if (cls == c) rank = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wc[c][wid] = __popcll(m);
    }
    __syncthreads();
    if (cls >= 0) {
        int32_t base = off[(int64_t)cls * n_tiles + tile];
        for (int w = 0; w < wid; ++w) base += wc[cls][w];
        bin_rows[base + rank] = v;
    }
}

// Slot sweep of one tile of kBlock nodes: one node per lane, 64 consecutive
// nodes per wave.  For every candidate slot whose in-edge bit is set, gather
// x at raw index i + off[s] (x lives in raw-index space, so neither col_idx
// nor an index remap is read).  A lane's in-edge bit for a slot is tested
// with one class comparison on a field of its record (see below), and the
// result is the execution mask of the slot's load, so lanes without the
// in-edge issue nothing.  The slot's offset goes into the load's scalar
// offset (the buffer base is moved down by the most negative offset so that
// every scalar offset is >= 0).  Slots run in ascending raw-index order, the
// order of the CSR rows, so the FP32 sum equals the one-lane-per-row CSR
// sweep's bit for bit.  The plain and the batched sweep both run this
// routine, so their results agree bit for bit.
struct SweepTile {
    const uint64_t *rec;         // node records
    const_ptr<int32_t> off;      // [k_pad] slot offsets, ascending (off[0] the most negative),
                                 // then [k_pad] byte offsets 4 (off[s] - off[0])
    const float *y_in, *x_in;
    float *y_out, *x_out;
    double *partials;
    double s, c, sd;
    int32_t n, k_slots, k_pad, x_bytes;
    LagTerms lt;   // lagged step only
};

// Slots per batch of the slot sweep.  All loads of a batch are issued before
// its first addition; because each load sits under its own execution-mask
// branch, the compiler cannot count the loads in flight and waits for the
// whole batch before adding, so a larger batch keeps more loads in flight per
// wave.  48 (three scalar loads of 16 offsets) measured fastest: 32 drains
// more often, 64 and 96 lower the occupancy (80 and 112 VGPRs).
constexpr int kSweepBatch = 48;

// The node of lane lt (0 <= lt < kBlock) of the tile: its new value, and its
// terms of the tile's three partial sums in ps, pr, pk (reduced by the
// caller).  LAG (the lagged step): the terms are added to ps, pr, pk.
template <int W, bool BUF, bool LAG = false>
__device__ __forceinline__ void sweep_tile_sums(const SweepTile &q, int32_t tile, int lt, double &ps, double &pr,
                                                double &pk) {
    // descriptor based at x_in + off[0] (<= x_in), so every slot's byte offset
    // 4 (off[s] - off[0]) is a non-negative scalar
    const int32_t off0 = q.off[0];
    const __amdgpu_buffer_rsrc_t xr =
        __builtin_amdgcn_make_buffer_rsrc((void *)(q.x_in + off0), (short)0, q.x_bytes, 0x00020000);
    const int32_t v = tile * kBlock + lt;
    const bool active = v < q.n;
    Record<W> r;
    float yin = 0.0f, yprev = 0.0f, gv = 0.0f;
    if (active) {
        r = load_record<W>(q.rec, v);
        // the node's own values are loaded with the record, ahead of the
        // gathers, so that their latency hides behind them; in every mode,
        // since loads under a branch on the mode make the compiler wait for
        // them before the gathers (8 us more per sweep at the large workload)
        yin = q.y_in[v];
        if (LAG) {
            yprev = q.lt.y_prev[v];
            gv = q.lt.g[v];
        }
    } else {
#pragma unroll
        for (int j = 0; j < W; ++j) r.w[j] = 0ull;
    }
    const int32_t i = r.raw();
    const uint32_t i4 = 4u * (uint32_t)i;
    // a wave past the last node (in the last tile) has nothing to gather
    const int32_t first = __builtin_amdgcn_readfirstlane(tile * kBlock + (lt & ~63));
    const bool live = first < q.n;
    const_ptr<int32_t> ob = q.off + q.k_pad;
    // The test of a node's in-edge bit for slot s is one class comparison:
    // its mask operand is a 10-bit field of the slot bits (slots 32j + 10t ..
    // 32j + 10t + 9 of word32 j), and its value operand a float whose IEEE
    // class is bit s mod 10 of the field (signalling NaN, quiet NaN, -inf,
    // -normal, -denormal, -0, +0, +denormal, +normal, +inf), against an AND
    // and a compare for a plain bit test.  The empty asm keeps the ten values
    // in SGPRs instead of re-materialising them per slot.
    uint32_t cls[10] = {0x7fa00000u, 0x7fc00000u, 0xff800000u, 0xbf800000u, 0x80000001u,
                        0x80000000u, 0x00000000u, 0x00000001u, 0x3f800000u, 0x7f800000u};
#pragma unroll
    for (int j = 0; j < 10; ++j) asm("" : "+s"(cls[j]));
    float acc = 0.0f;
    asm("" : "+v"(acc));   // keeps the first addition out of the first slot's branch
    constexpr int kB = kSweepBatch;
#pragma unroll
    for (int b = 0; b < (64 * W + kB - 1) / kB; ++b) {
        if (kB * b >= q.k_slots || !live) break;
        float val[kB];
#pragma unroll
        for (int h = 0; h < kB / 16; ++h) {
            // 16 offsets in one wide scalar load, ahead of the gathers (the
            // table is padded past the last batch)
            typedef int32_t i32x16 __attribute__((ext_vector_type(16)));
            const i32x16 o = *(const __attribute__((address_space(4))) i32x16 *)(
                (BUF ? ob : q.off) + kB * b + 16 * h);
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                const int u = 16 * h + t, sl = kB * b + u;
                val[u] = 0.0f;
                if (sl < 64 * W) {
                    // word32 of the slot; bits above slot k carry out_deg and
                    // the raw index and are masked off
                    const uint32_t wd = (uint32_t)(r.w[sl >> 6] >> (32 * ((sl >> 5) & 1))) &
                                        batch_mask(sl >> 5, q.k_slots);
                    // lanes without the in-edge skip the load (execution mask)
                    if (__builtin_amdgcn_classf(__uint_as_float(cls[(sl & 31) % 10]),
                                                (int)(wd >> (10 * ((sl & 31) / 10))))) {
                        if (BUF)
                            val[u] = __int_as_float(__builtin_amdgcn_raw_buffer_load_b32(xr, i4, (uint32_t)o[t], 0));
                        else
                            val[u] = q.x_in[i + o[t]];
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) acc += val[u];
    }
    if (LAG) {
        if (active) {
            const int32_t deg = r.out_deg();
            const float yf = lag_node(q.lt, v, acc, yin, yprev, gv, deg, ps, pr, pk);
            q.y_out[v] = yf;
            q.x_out[i] = deg > 0 ? yf / (float)deg : 0.0f;
        }
        return;
    }
    ps = pr = pk = 0.0;
    if (active) {
        const float yf = (float)(q.sd * (double)acc + q.c);
        q.y_out[v] = yf;
        q.x_out[i] = r.out_deg() > 0 ? yf / (float)r.out_deg() : 0.0f;
        ps = (double)yf;
        pr = fabs((double)yf - q.s * (double)yin);
        if (r.out_deg() == 0) pk = (double)yf;
    }
}

template <int W, bool BUF>
__device__ __forceinline__ void sweep_tile(const SweepTile &q, int32_t tile) {
    double ps, pr, pk;
    sweep_tile_sums<W, BUF>(q, tile, (int)threadIdx.x, ps, pr, pk);
    write_partials(q.partials, tile, ps, pr, pk);
}

// LAG: the lagged step (see lag_step); the workgroup's terms make one
// triple: each thread adds its nodes' terms over its tiles in LDS (so that no
// FP64 sums stay live in registers across the gathers), then one fixed tree
// reduces the threads' sums.
template <int W, bool BUF, bool LAG>
__global__ __launch_bounds__(kBlock) void k_pr_iter_slots(PrArgs a) {
    const PrState *st = a.st;
    if (st->done) return;
    if (LAG) {
        if (blockIdx.x == 0 && a.sweep >= 1) lag_step(a);
        if (!lag_has_tiles(a)) return;
    }
    const int32_t k = LAG ? a.sweep : st->k;
    SweepTile q;
    q.rec = a.rec;
    q.off = to_const(a.off);
    q.y_in = a.y[LAG ? k % 3 : k & 1];
    q.x_in = a.x[k & 1];
    q.y_out = a.y[LAG ? (k + 1) % 3 : (k + 1) & 1];
    q.x_out = a.x[(k + 1) & 1];
    q.partials = a.partials;
    if (LAG) {
        q.s = q.c = q.sd = 0.0;
        q.lt = lag_terms(a);
    } else {
        q.s = st->s;
        q.c = st->c;
        q.sd = q.s * a.d;
    }
    q.n = a.n;
    q.k_slots = a.k_slots;
    q.k_pad = a.k_pad;
    q.x_bytes = a.x_bytes;
    const TileWalk w((a.n + kBlock - 1) / kBlock);
    if (LAG) {
        // each thread's running sums live in LDS between its tiles
        __shared__ double sums[3][kBlock];
        const int lt = (int)threadIdx.x;
        sums[0][lt] = sums[1][lt] = sums[2][lt] = 0.0;
        for (int32_t t = w.first; t < w.end; t += w.step) {
            const int32_t stop = peek_stop(a.st);   // its latency hides behind the tile
            double ps = 0.0, pr = 0.0, pk = 0.0;
            sweep_tile_sums<W, BUF, true>(q, t, lt, ps, pr, pk);
            sums[0][lt] += ps;
            sums[1][lt] += pr;
            sums[2][lt] += pk;
            if (stop) break;   // per wave: this loop has no barrier
        }
        write_lag_partials(a, sums[0][lt], sums[1][lt], sums[2][lt]);
    } else {
        for (int32_t t = w.first; t < w.end; t += w.step) sweep_tile<W, BUF>(q, t);
    }
}

// ---------------------------------------------------------------------------
// Batched power iteration: many FFGs (members) swept together.  A tile list
// names (member, tile) pairs; each tile reads its member's descriptor through
// the scalar unit and writes its own three FP64 partial sums, so a member's
// result does not depend on which other members share the launch.  A member
// whose stop flag is set is skipped.

template <int W, bool BUF>
__global__ __launch_bounds__(kBlock) void k_batch_sweep(const BatchMember *__restrict__ members,
                                                        const TileRef *__restrict__ tiles,
                                                        const int32_t *__restrict__ range_dev) {
    // the list's start and length are read from device memory, so a captured
    // launch stays valid while members join and leave between replays
    const int32_t begin = to_const(range_dev)[0], count = to_const(range_dev)[1];
    const TileWalk w(count);
    const_ptr<TileRef> tl = to_const(tiles) + begin;
    for (int32_t t = w.first; t < w.end; t += w.step) {
        const int32_t member = tl[t].member, tile = tl[t].tile;
        const_ptr<BatchMember> m = to_const(members) + member;
        const_ptr<PrState> st = to_const(m->st);
        if (st->done) continue;
        const int32_t k = st->k;
        SweepTile q;
        q.rec = m->rec;
        q.off = to_const(m->off);
        q.y_in = m->y[k & 1];
        q.x_in = m->x[k & 1];
        q.y_out = m->y[(k + 1) & 1];
        q.x_out = m->x[(k + 1) & 1];
        q.partials = m->partials;
        q.s = st->s;
        q.c = st->c;
        q.sd = q.s * m->d;
        q.n = m->n;
        q.k_slots = m->k_slots;
        q.k_pad = m->k_pad;
        q.x_bytes = m->x_bytes;
        sweep_tile<W, BUF>(q, tile);
    }
}

// Binned members: each listed (member, tile) is a tile of the member's bin
// table, swept as by k_pr_iter_binned.
__global__ __launch_bounds__(kBlock) void k_batch_sweep_binned(const BatchMember *__restrict__ members,
                                                               const TileRef *__restrict__ tiles,
                                                               const int32_t *__restrict__ range_dev) {
    const int32_t begin = to_const(range_dev)[0], count = to_const(range_dev)[1];
    const TileWalk w(count);
    const_ptr<TileRef> tl = to_const(tiles) + begin;
    for (int32_t t = w.first; t < w.end; t += w.step) {
        const int32_t member = tl[t].member, tile = tl[t].tile;
        const_ptr<BatchMember> m = to_const(members) + member;
        const_ptr<PrState> st = to_const(m->st);
        if (st->done) continue;
        const int32_t k = st->k;
        BinSweep q;
        q.row_ptr = m->row_ptr;
        q.col_idx = m->col_idx;
        q.out_deg = m->out_deg;
        q.rows = m->bin_rows;
        q.y_in = m->y[k & 1];
        q.x_in = m->x[k & 1];
        q.y_out = m->y[(k + 1) & 1];
        q.x_out = m->x[(k + 1) & 1];
        q.s = st->s;
        q.c = st->c;
        q.sd = q.s * m->d;
        double ps = 0.0, pr = 0.0, pk = 0.0;
        binned_tile<false>(q, &m->bins, tile, ps, pr, pk);
        write_partials(m->partials, tile, ps, pr, pk);
    }
}

// Initial iterate r = 1/N of every listed tile, with its partial sums.
__global__ __launch_bounds__(kBlock) void k_batch_init(const BatchMember *__restrict__ members,
                                                       const TileRef *__restrict__ tiles, int32_t n_tiles) {
    for (int32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const TileRef tr = tiles[t];
        const BatchMember &m = members[tr.member];
        init_tile(tr.tile, m.n, m.out_deg, m.xmap, m.y[0], m.x[0], m.partials);
    }
}

// One workgroup per listed member (grid-stride over the list, whose length
// is read from device memory): reduce its tiles' partial sums and set up its
// next step, exactly as for a single space.
template <bool FIRST>
__global__ __launch_bounds__(kFinishBlock) void k_batch_finish(const BatchMember *__restrict__ members,
                                                         const int32_t *__restrict__ member_ids,
                                                         const int32_t *__restrict__ n_members_dev) {
    const int32_t n_members = *to_const(n_members_dev);
    for (int32_t j = blockIdx.x; j < n_members; j += gridDim.x) {
        const BatchMember &m = members[member_ids[j]];
        if (!FIRST && m.st->done) continue;   // uniform per workgroup
        finish_step(m.st, m.partials, FIRST ? m.n_tiles : m.n_parts, m.d, m.tol, m.max_iter, m.n, FIRST);
        __syncthreads();                       // block_sum3's LDS is reused by the next member
    }
}

// Small members (at most kSmallTiles tiles): one workgroup of kFinishBlock
// threads runs a member's sweeps and steps back to back, up to max_sweeps or
// until it stops, with workgroup barriers instead of launches between them.
// The four groups of kBlock threads sweep four tiles at a time; each group
// reduces its tile's partial sums in the order of block_sum3 (wave sums, then
// the four waves in order), and the step is finish_step itself, so a
// member's ranks equal those of the plain slot sweep bit for bit.  Thread 0
// (which writes the state in finish_step) hands the stop flag, k, s and c to
// the workgroup through LDS, so every wave takes the same branches.
constexpr int kGroups = kFinishBlock / kBlock;

template <int W>
__global__ __launch_bounds__(kFinishBlock) void k_batch_small(const BatchMember *__restrict__ members,
                                                              const int32_t *__restrict__ member_ids,
                                                              int32_t n_members, int32_t max_sweeps) {
    __shared__ double part[kGroups][3][kBlock / 64];
    __shared__ int32_t sh_done, sh_k;
    __shared__ double sh_s, sh_c;
    const int g = threadIdx.x / kBlock, lt = threadIdx.x % kBlock;
    const int lane = threadIdx.x & 63, wl = lt >> 6;
    for (int32_t j = blockIdx.x; j < n_members; j += gridDim.x) {
        const_ptr<BatchMember> m = to_const(members) + member_ids[j];
        PrState *st = m->st;
        for (int32_t sweep = 0; sweep < max_sweeps; ++sweep) {
            if (threadIdx.x == 0) {
                sh_done = st->done;
                sh_k = st->k;
                sh_s = st->s;
                sh_c = st->c;
            }
            __syncthreads();
            if (sh_done) break;               // uniform
            const int32_t k = sh_k;
            SweepTile q;
            q.rec = m->rec;
            q.off = to_const(m->off);
            q.y_in = m->y[k & 1];
            q.x_in = m->x[k & 1];
            q.y_out = m->y[(k + 1) & 1];
            q.x_out = m->x[(k + 1) & 1];
            q.partials = m->partials;
            q.s = sh_s;
            q.c = sh_c;
            q.sd = q.s * m->d;
            q.n = m->n;
            q.k_slots = m->k_slots;
            q.k_pad = m->k_pad;
            q.x_bytes = m->x_bytes;
            const int32_t n_tiles = m->n_tiles;
            for (int32_t t0 = 0; t0 < n_tiles; t0 += kGroups) {
                const int32_t tile = t0 + g;      // a group past the last tile only joins the barriers
                double ps = 0.0, pr = 0.0, pk = 0.0;
                if (tile < n_tiles) sweep_tile_sums<W, true>(q, tile, lt, ps, pr, pk);
                ps = wave_sum(ps);
                pr = wave_sum(pr);
                pk = wave_sum(pk);
                if (lane == 0) {
                    part[g][0][wl] = ps;
                    part[g][1][wl] = pr;
                    part[g][2][wl] = pk;
                }
                __syncthreads();
                if (lt == 0 && tile < n_tiles) {
                    double a = part[g][0][0], b = part[g][1][0], c = part[g][2][0];
#pragma unroll
                    for (int w = 1; w < kBlock / 64; ++w) {
                        a += part[g][0][w];
                        b += part[g][1][w];
                        c += part[g][2][w];
                    }
                    double *pp = m->partials + 3 * (int64_t)tile;
                    pp[0] = a;
                    pp[1] = b;
                    pp[2] = c;
                }
                __syncthreads();                  // part is reused; the partials are visible
            }
            finish_step(st, m->partials, n_tiles, m->d, m->tol, m->max_iter, m->n, false);
        }
        __syncthreads();                          // sh_* are rewritten for the next member
    }
}

// Ranks r = y * s into the member's output for every listed tile.
__global__ __launch_bounds__(kBlock) void k_batch_output(const BatchMember *__restrict__ members,
                                                         const TileRef *__restrict__ tiles, int32_t n_tiles) {
    for (int32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const TileRef tr = tiles[t];
        const BatchMember &m = members[tr.member];
        const int32_t v = tr.tile * kBlock + threadIdx.x;
        if (v < m.n) m.out_pagerank[v] = (double)m.y[m.st->k & 1][v] * m.st->s;
    }
}

// One workgroup per listed member: copy its minima out, C_p sums (as k_score),
// and a snapshot of its state into states_out[blockIdx.x].
__global__ __launch_bounds__(kBlock) void k_batch_score(const BatchMember *__restrict__ members,
                                                        const int32_t *__restrict__ member_ids,
                                                        PrState *__restrict__ states_out) {
    const BatchMember &m = members[member_ids[blockIdx.x]];
    PrState *st = m.st;
    double num = 0.0, den = 0.0;
    for (int32_t j = threadIdx.x; j < m.m; j += kBlock) {
        const int32_t v = m.minima[j];
        m.out_minima[j] = v;
        const double r = m.out_pagerank[v];
        den += r;
        if ((double)m.fit_c[v] <= m.threshold) num += r;
    }
    num = block_sum(num);
    den = block_sum(den);
    if (threadIdx.x == 0) {
        st->score_num = num;
        st->score_den = den;
        states_out[blockIdx.x] = *st;
    }
}

// C_p curve (Sec. VII-B, eq. 3, for many p): workgroup j sums the ranks of
// the minima with (double) f <= thresholds[j] and of all minima, in FP64.
__global__ __launch_bounds__(kBlock) void k_score_curve(const double *__restrict__ pagerank,
                                                        const int32_t *__restrict__ minima, int32_t m,
                                                        const float *__restrict__ fit_c,
                                                        const double *__restrict__ thresholds,
                                                        double *__restrict__ num_den) {
    const double t = thresholds[blockIdx.x];
    double num = 0.0, den = 0.0;
    for (int32_t j = threadIdx.x; j < m; j += kBlock) {
        const int32_t v = minima[j];
        const double r = pagerank[v];
        den += r;
        if ((double)fit_c[v] <= t) num += r;
    }
    num = block_sum(num);
    den = block_sum(den);
    if (threadIdx.x == 0) {
        num_den[2 * blockIdx.x] = num;
        num_den[2 * blockIdx.x + 1] = den;
    }
}

// Fraction of optimal fitness f_opt / f(m) of every local minimum, and its
// histogram over n_bins equal bins of [0, 1] (integer counts, exact).
__global__ __launch_bounds__(kBlock) void k_naive(const int32_t *__restrict__ minima, int32_t m,
                                                  const float *__restrict__ fit_c, float f_opt,
                                                  double *__restrict__ ratio, int32_t n_bins,
                                                  uint32_t *__restrict__ hist) {
    for (int32_t j = blockIdx.x * kBlock + threadIdx.x; j < m; j += gridDim.x * kBlock) {
        const double q = (double)f_opt / (double)fit_c[minima[j]];
        ratio[j] = q;
        const int32_t bin = min((int32_t)floor(q * (double)n_bins), n_bins - 1);
        atomicAdd(&hist[bin], 1u);
    }
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int32_t n, uint32_t value) {
    for (int32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) p[j] = value;
}

__global__ void k_batch_states(const BatchMember *__restrict__ members, const int32_t *__restrict__ member_ids,
                               int32_t n_members, PrState *__restrict__ states_out) {
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n_members) states_out[j] = *members[member_ids[j]].st;
}

__global__ __launch_bounds__(kBlock) void k_pr_output(PrArgs a, double *__restrict__ pagerank) {
    const PrState *st = a.st;
    if (a.lag) {
        // r = w + gamma, scaled to sum 1
        const float *__restrict__ y = a.y[st->out_buf];
        const double g = st->out_gamma, s = 1.0 / st->out_sigma;
        for (int32_t v = blockIdx.x * kBlock + threadIdx.x; v < a.n; v += gridDim.x * kBlock)
            pagerank[v] = ((double)y[v] + g) * s;
        return;
    }
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


// The slot sweep kernel for W record words, with out-of-range buffer loads
// when the x vector's byte size leaves room for the out-of-range offset.
template <int W>
const void *slot_sweep_fn(const PrArgs &a) {
    if (a.lag)
        return a.x_bytes > 0 ? (const void *)k_pr_iter_slots<W, true, true> : (const void *)k_pr_iter_slots<W, false, true>;
    return a.x_bytes > 0 ? (const void *)k_pr_iter_slots<W, true, false> : (const void *)k_pr_iter_slots<W, false, false>;
}

const void *slot_sweep_kernel(const PrArgs &a, int words) {
    switch (words) {
        case 1: return slot_sweep_fn<1>(a);
        case 2: return slot_sweep_fn<2>(a);
        case 3: return slot_sweep_fn<3>(a);
        case 4: return slot_sweep_fn<4>(a);
        case 5: return slot_sweep_fn<5>(a);
        default: return nullptr;
    }
}

template <bool LAG>
const void *csr_sweep_fn(int lanes) {
    switch (lanes) {
        case 1: return (const void *)k_pr_iter_csr<1, LAG>;
        case 2: return (const void *)k_pr_iter_csr<2, LAG>;
        case 4: return (const void *)k_pr_iter_csr<4, LAG>;
        case 8: return (const void *)k_pr_iter_csr<8, LAG>;
        case 16: return (const void *)k_pr_iter_csr<16, LAG>;
        case 32: return (const void *)k_pr_iter_csr<32, LAG>;
        case 64: return (const void *)k_pr_iter_csr<64, LAG>;
        default: return nullptr;
    }
}

const void *csr_sweep_kernel(const PrArgs &a, int lanes) {
    return a.lag ? csr_sweep_fn<true>(lanes) : csr_sweep_fn<false>(lanes);
}

const void *binned_sweep_kernel(bool lag) {
    return lag ? (const void *)k_pr_iter_binned<true> : (const void *)k_pr_iter_binned<false>;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers.

hipError_t launch_compact_single(const float *fit, int32_t n_raw, int32_t *tile_cnt, float *tile_min,
                                 int32_t *tile_bad, int32_t *remap, int32_t *valid_raw, float *fit_c,
                                 BuildSizes *sizes, hipStream_t stream) {
    const int32_t tiles = (n_raw + kSingleTile - 1) / kSingleTile;
    if (((uintptr_t)fit & 15u) == 0) {
        hipLaunchKernelGGL(k_compact_tiles<true>, dim3(tiles), dim3(kBlock), 0, stream, fit, n_raw, tile_cnt, tile_min,
                           tile_bad);
        hipLaunchKernelGGL(k_compact_place<true>, dim3(tiles), dim3(kBlock), 0, stream, fit, n_raw, tiles, tile_cnt,
                           tile_min, tile_bad, remap, valid_raw, fit_c, sizes);
    } else {
        hipLaunchKernelGGL(k_compact_tiles<false>, dim3(tiles), dim3(kBlock), 0, stream, fit, n_raw, tile_cnt,
                           tile_min, tile_bad);
        hipLaunchKernelGGL(k_compact_place<false>, dim3(tiles), dim3(kBlock), 0, stream, fit, n_raw, tiles, tile_cnt,
                           tile_min, tile_bad, remap, valid_raw, fit_c, sizes);
    }
    return hipGetLastError();
}

hipError_t launch_seg_compact(const SegBuild *segs, const SegTile *tiles, int32_t n_tiles, const int32_t *ids,
                              int32_t n_ids, hipStream_t stream) {
    if (n_tiles <= 0 || n_ids <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_compact_count, dim3(n_tiles), dim3(kBlock), 0, stream, segs, tiles);
    hipLaunchKernelGGL(k_seg_compact_scan, dim3(n_ids), dim3(kBlock), 0, stream, segs, ids);
    hipLaunchKernelGGL(k_seg_compact_write, dim3(n_tiles), dim3(kBlock), 0, stream, segs, tiles);
    return hipGetLastError();
}

template <int W>
static const void *seg_degree_kernel(bool buf) {
    return buf ? (const void *)k_seg_degree<W, true> : (const void *)k_seg_degree<W, false>;
}

template <int W>
static const void *seg_fill_kernel(bool buf) {
    return buf ? (const void *)k_seg_fill<W, true> : (const void *)k_seg_fill<W, false>;
}

static hipError_t launch_seg_tiles(const void *fn, const SegBuild *segs, const SegTile *tiles, int32_t n_tiles,
                                   hipStream_t stream) {
    if (!fn) return hipErrorInvalidValue;
    if (n_tiles <= 0) return hipSuccess;
    void *args[] = {(void *)&segs, (void *)&tiles};
    return hipLaunchKernel(fn, dim3(n_tiles), dim3(kBlock), args, 0, stream);
}

hipError_t launch_seg_degree(const SegBuild *segs, const SegTile *tiles, int32_t n_tiles, int words, bool buf,
                             hipStream_t stream) {
    const void *fn = nullptr;
    switch (words) {
        case 1: fn = seg_degree_kernel<1>(buf); break;
        case 2: fn = seg_degree_kernel<2>(buf); break;
        case 3: fn = seg_degree_kernel<3>(buf); break;
        case 4: fn = seg_degree_kernel<4>(buf); break;
        case 5: fn = seg_degree_kernel<5>(buf); break;
        default: break;
    }
    return launch_seg_tiles(fn, segs, tiles, n_tiles, stream);
}

hipError_t launch_seg_degree_scan(const SegBuild *segs, const int32_t *ids, int32_t n_ids, hipStream_t stream) {
    if (n_ids <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_seg_degree_scan, dim3(n_ids), dim3(kBlock), 0, stream, segs, ids);
    return hipGetLastError();
}

hipError_t launch_seg_fill(const SegBuild *segs, const SegTile *tiles, int32_t n_tiles, int words, bool buf,
                           hipStream_t stream) {
    const void *fn = nullptr;
    switch (words) {
        case 1: fn = seg_fill_kernel<1>(buf); break;
        case 2: fn = seg_fill_kernel<2>(buf); break;
        case 3: fn = seg_fill_kernel<3>(buf); break;
        case 4: fn = seg_fill_kernel<4>(buf); break;
        case 5: fn = seg_fill_kernel<5>(buf); break;
        default: break;
    }
    return launch_seg_tiles(fn, segs, tiles, n_tiles, stream);
}

template <int W>
static const void *degree_slots_kernel(bool buf) {
    return buf ? (const void *)k_degree_slots<W, true> : (const void *)k_degree_slots<W, false>;
}

hipError_t launch_degree(const SpaceDesc &sp, const SlotTable &sl, int adjacent, const float *fit,
                         const int32_t *valid_raw, int32_t n, int32_t *in_deg, int32_t *out_deg,
                         uint64_t *rec, uint64_t *presence, int32_t *off_table, int32_t k_pad,
                         int64_t *tile_e, int32_t *tile_m, int64_t *tile_eoff, int32_t *tile_moff,
                         BuildSizes *sizes, hipStream_t stream) {
    const int32_t tiles = (n + kBlock - 1) / kBlock;
    if (sl.words > 0) {
        // buffer loads of the fitness need 4 n_raw < 2^31 (room for the out-of-range bit)
        const bool buf = 4 * (int64_t)sp.n_raw < (int64_t(1) << 31);
        const int32_t fit_bytes = buf ? 4 * sp.n_raw : 0;
        const void *fn = nullptr;
        switch (sl.words) {
            case 1: fn = degree_slots_kernel<1>(buf); break;
            case 2: fn = degree_slots_kernel<2>(buf); break;
            case 3: fn = degree_slots_kernel<3>(buf); break;
            case 4: fn = degree_slots_kernel<4>(buf); break;
            case 5: fn = degree_slots_kernel<5>(buf); break;
            default: return hipErrorInvalidValue;
        }
        SegBuild g{};
        g.sp = sp;
        g.sl = sl;
        g.fit = fit;
        g.fit_bytes = fit_bytes;
        g.valid_raw = const_cast<int32_t *>(valid_raw);
        g.n = n;
        g.in_deg = in_deg;
        g.out_deg = out_deg;
        g.rec = rec;
        g.presence = presence;
        g.off_table = off_table;
        g.k_pad = k_pad;
        g.tile_e = tile_e;
        g.tile_m = tile_m;
        g.sizes = sizes;
        void *args[] = {(void *)&g};
        hipError_t e = hipLaunchKernel(fn, dim3(tiles), dim3(kBlock), args, 0, stream);
        if (e != hipSuccess) return e;
    }
    switch (sl.words) {
        case 1: case 2: case 3: case 4: case 5: break;
        case 0:
            if (adjacent)
                hipLaunchKernelGGL(k_degree_generic<true>, dim3(tiles), dim3(kBlock), 0, stream, sp, fit, valid_raw,
                                   n, in_deg, out_deg, tile_e, tile_m, sizes);
            else
                hipLaunchKernelGGL(k_degree_generic<false>, dim3(tiles), dim3(kBlock), 0, stream, sp, fit, valid_raw,
                                   n, in_deg, out_deg, tile_e, tile_m, sizes);
            break;
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_degree_scan, dim3(1), dim3(kFinishBlock), 0, stream, tile_e, tile_m, tiles,
                       tile_eoff, tile_moff, sizes);
    return hipGetLastError();
}

template <int W>
static const void *fill_slots_kernel(bool buf) {
    return buf ? (const void *)k_fill_slots<W, true> : (const void *)k_fill_slots<W, false>;
}

hipError_t launch_fill(const SpaceDesc &sp, const SlotTable &sl, int adjacent, const float *fit,
                       const int32_t *valid_raw, const int32_t *remap, const uint64_t *rec,
                       const uint64_t *presence, int32_t n, int32_t n_edges, const int32_t *in_deg,
                       const int32_t *out_deg, const int64_t *tile_eoff, const int32_t *tile_moff,
                       int32_t *row_ptr, int32_t *col_idx, int32_t *minima, hipStream_t stream) {
    const int32_t tiles = (n + kBlock - 1) / kBlock;
    if (sl.words > 0) {
        // buffer loads of remap need 4 n_raw < 2^31 (room for the out-of-range bit)
        const bool buf = 4 * (int64_t)sp.n_raw < (int64_t(1) << 31);
        const int32_t remap_bytes = buf ? 4 * sp.n_raw : 0;
        const void *fn = nullptr;
        switch (sl.words) {
            case 1: fn = fill_slots_kernel<1>(buf); break;
            case 2: fn = fill_slots_kernel<2>(buf); break;
            case 3: fn = fill_slots_kernel<3>(buf); break;
            case 4: fn = fill_slots_kernel<4>(buf); break;
            case 5: fn = fill_slots_kernel<5>(buf); break;
            default: return hipErrorInvalidValue;
        }
        SegBuild g{};
        g.sl = sl;
        g.remap = const_cast<int32_t *>(remap);
        g.remap_bytes = remap_bytes;
        g.rec = const_cast<uint64_t *>(rec);
        g.presence = const_cast<uint64_t *>(presence);
        g.n = n;
        g.n_edges = n_edges;
        g.in_deg = const_cast<int32_t *>(in_deg);
        g.out_deg = const_cast<int32_t *>(out_deg);
        g.tile_eoff = const_cast<int64_t *>(tile_eoff);
        g.tile_moff = const_cast<int32_t *>(tile_moff);
        g.row_ptr = row_ptr;
        g.col_idx = col_idx;
        g.minima = minima;
        void *args[] = {(void *)&g};
        return hipLaunchKernel(fn, dim3(tiles), dim3(kBlock), args, 0, stream);
    }
    switch (sl.words) {
        case 0:
            if (adjacent)
                hipLaunchKernelGGL(k_fill_generic<true>, dim3(tiles), dim3(kBlock), 0, stream, sp, fit, valid_raw, remap,
                                   n, n_edges, in_deg, out_deg, tile_eoff, tile_moff, row_ptr, col_idx, minima);
            else
                hipLaunchKernelGGL(k_fill_generic<false>, dim3(tiles), dim3(kBlock), 0, stream, sp, fit, valid_raw, remap,
                                   n, n_edges, in_deg, out_deg, tile_eoff, tile_moff, row_ptr, col_idx, minima);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pr_init(const PrArgs &a, int grid, hipStream_t stream) {
    if (a.lag) {
        hipLaunchKernelGGL(k_pr_init_lag, dim3(grid), dim3(kBlock), 0, stream, a);
        return hipGetLastError();
    }
    const int32_t n_tiles = (a.n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_pr_init, dim3(grid), dim3(kBlock), 0, stream, a);
    hipLaunchKernelGGL(k_pr_finish<true>, dim3(1), dim3(kFinishBlock), 0, stream, a, n_tiles);
    return hipGetLastError();
}

hipError_t pr_iter_blocks_per_cu(const PrArgs &a, const SpaceDesc &sp, const SlotTable &sl, int lanes,
                                 int *blocks) {
    (void)sp;
    if (a.kind == kSweepBinned) return pr_binned_blocks_per_cu(blocks, a.lag != 0);
    const void *fn = a.kind == kSweepSlots ? slot_sweep_kernel(a, sl.words) : csr_sweep_kernel(a, lanes);
    if (!fn) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kBlock, 0);
}

hipError_t launch_pr_sweep_binned(const PrArgs &a, const BinTable &t, int grid, hipStream_t stream) {
    if (t.tiles <= 0) return hipSuccess;
    PrArgs b = a;
    b.bins = t;
    void *args[] = {(void *)&b};
    return hipLaunchKernel(binned_sweep_kernel(a.lag != 0), dim3(grid), dim3(kBlock), args, 0, stream);
}

hipError_t pr_binned_blocks_per_cu(int *blocks, bool lag) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, binned_sweep_kernel(lag), kBlock, 0);
}

hipError_t launch_bin_rows(const int32_t *row_ptr, int32_t n, const int8_t *class_of_dev, int32_t *cnt,
                           int32_t *off, int32_t *totals, int32_t *bin_rows, hipStream_t stream) {
    const int32_t n_tiles = (n + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_bin_count, dim3(n_tiles), dim3(kBlock), 0, stream, row_ptr, n, class_of_dev, cnt, n_tiles);
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(kBlock), 0, stream, cnt, off, totals, n_tiles);
    hipLaunchKernelGGL(k_bin_write, dim3(n_tiles), dim3(kBlock), 0, stream, row_ptr, n, class_of_dev, off, n_tiles,
                       bin_rows);
    return hipGetLastError();
}

hipError_t launch_pr_sweep(const PrArgs &a, const SlotTable &sl, int lanes, int grid, hipStream_t stream) {
    if (a.kind == kSweepBinned) return launch_pr_sweep_binned(a, a.bins, grid, stream);
    const void *fn = a.kind == kSweepSlots ? slot_sweep_kernel(a, sl.words) : csr_sweep_kernel(a, lanes);
    if (!fn) return hipErrorInvalidValue;
    void *args[] = {(void *)&a};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, 0, stream);
}

hipError_t launch_pr_step(const PrArgs &a, int grid, hipStream_t stream) {
    if (a.lag) return hipSuccess;   // the next sweep does the step
    // partial sums: one triple per tile (slot sweep, binned sweep) or per
    // workgroup (CSR sweep)
    const int32_t count = a.kind == kSweepSlots ? (a.n + kBlock - 1) / kBlock
                          : a.kind == kSweepBinned ? a.bins.tiles : grid;
    hipLaunchKernelGGL(k_pr_finish<false>, dim3(1), dim3(kFinishBlock), 0, stream, a, count);
    return hipGetLastError();
}

hipError_t launch_pr_iter(const PrArgs &a, const SpaceDesc &sp, const SlotTable &sl, int lanes,
                          int grid, hipStream_t stream) {
    (void)sp;
    hipError_t e = launch_pr_sweep(a, sl, lanes, grid, stream);
    if (e != hipSuccess) return e;
    return launch_pr_step(a, grid, stream);
}

hipError_t launch_pr_output(const PrArgs &a, double *pagerank, hipStream_t stream) {
    const int grid = (int)(((int64_t)a.n + kBlock - 1) / kBlock < 4096 ? ((int64_t)a.n + kBlock - 1) / kBlock : 4096);
    hipLaunchKernelGGL(k_pr_output, dim3(grid), dim3(kBlock), 0, stream, a, pagerank);
    return hipGetLastError();
}

hipError_t launch_score(const double *pagerank, const int32_t *minima, int32_t m,
                        const float *fit_c, double threshold, PrState *st, hipStream_t stream) {
    hipLaunchKernelGGL(k_score, dim3(1), dim3(kBlock), 0, stream, pagerank, minima, m, fit_c,
                       threshold, st);
    return hipGetLastError();
}

hipError_t launch_score_curve(const double *pagerank, const int32_t *minima, int32_t m, const float *fit_c,
                              const double *thresholds, int32_t n, double *num_den, hipStream_t stream) {
    if (n > 0)
        hipLaunchKernelGGL(k_score_curve, dim3(n), dim3(kBlock), 0, stream, pagerank, minima, m, fit_c, thresholds,
                           num_den);
    return hipGetLastError();
}

hipError_t launch_naive(const int32_t *minima, int32_t m, const float *fit_c, float f_opt, double *ratio,
                        int32_t n_bins, uint32_t *hist, hipStream_t stream) {
    hipLaunchKernelGGL(k_fill_u32, dim3((n_bins + 255) / 256), dim3(256), 0, stream, hist, n_bins, 0u);
    if (m > 0)
        hipLaunchKernelGGL(k_naive, dim3(std::min<int32_t>((m + kBlock - 1) / kBlock, 1024)), dim3(kBlock), 0,
                           stream, minima, m, fit_c, f_opt, ratio, n_bins, hist);
    return hipGetLastError();
}

hipError_t launch_batch_init(const BatchMember *members, const TileRef *tiles, int32_t n_tiles,
                             const int32_t *member_ids, int32_t n_members, const int32_t *n_members_dev,
                             hipStream_t stream) {
    if (n_tiles > 0)
        hipLaunchKernelGGL(k_batch_init, dim3(std::min<int32_t>(n_tiles, 8192)), dim3(kBlock), 0, stream, members,
                           tiles, n_tiles);
    if (n_members > 0)
        hipLaunchKernelGGL(k_batch_finish<true>, dim3(std::min<int32_t>(n_members, kMaxFinishGrid)), dim3(kFinishBlock), 0,
                           stream, members, member_ids, n_members_dev);
    return hipGetLastError();
}

static const void *batch_sweep_kernel(int words) {
    switch (words) {
        case 1: return (const void *)k_batch_sweep<1, true>;
        case 2: return (const void *)k_batch_sweep<2, true>;
        case 3: return (const void *)k_batch_sweep<3, true>;
        case 4: return (const void *)k_batch_sweep<4, true>;
        case 5: return (const void *)k_batch_sweep<5, true>;
        default: return nullptr;
    }
}

hipError_t launch_batch_sweep_binned(const BatchMember *members, const TileRef *tiles, const int32_t *range_dev,
                                     int grid, hipStream_t stream) {
    hipLaunchKernelGGL(k_batch_sweep_binned, dim3(grid), dim3(kBlock), 0, stream, members, tiles, range_dev);
    return hipGetLastError();
}

hipError_t batch_sweep_binned_blocks_per_cu(int *blocks) {
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void *)k_batch_sweep_binned, kBlock, 0);
}

hipError_t batch_sweep_blocks_per_cu(int words, int *blocks) {
    const void *fn = batch_sweep_kernel(words);
    if (!fn) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kBlock, 0);
}

hipError_t launch_batch_sweep(const BatchMember *members, const TileRef *tiles, const int32_t *range_dev,
                              int words, int grid, hipStream_t stream) {
    const void *fn = batch_sweep_kernel(words);
    if (!fn) return hipErrorInvalidValue;
    void *args[] = {(void *)&members, (void *)&tiles, (void *)&range_dev};
    return hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, 0, stream);
}

static const void *batch_small_kernel(int words) {
    switch (words) {
        case 1: return (const void *)k_batch_small<1>;
        case 2: return (const void *)k_batch_small<2>;
        case 3: return (const void *)k_batch_small<3>;
        case 4: return (const void *)k_batch_small<4>;
        case 5: return (const void *)k_batch_small<5>;
        default: return nullptr;
    }
}

hipError_t launch_batch_small(const BatchMember *members, const int32_t *member_ids, int32_t n_members, int words,
                              int32_t max_sweeps, int grid, hipStream_t stream) {
    const void *fn = batch_small_kernel(words);
    if (!fn) return hipErrorInvalidValue;
    if (n_members <= 0 || max_sweeps <= 0) return hipSuccess;
    void *args[] = {(void *)&members, (void *)&member_ids, (void *)&n_members, (void *)&max_sweeps};
    return hipLaunchKernel(fn, dim3(grid), dim3(kFinishBlock), args, 0, stream);
}

hipError_t launch_batch_finish(const BatchMember *members, const int32_t *member_ids, const int32_t *n_members_dev,
                               int grid, hipStream_t stream) {
    hipLaunchKernelGGL(k_batch_finish<false>, dim3(grid), dim3(kFinishBlock), 0, stream, members, member_ids,
                       n_members_dev);
    return hipGetLastError();
}

hipError_t launch_batch_output(const BatchMember *members, const TileRef *tiles, int32_t n_tiles,
                               const int32_t *member_ids, int32_t n_members, PrState *states_out,
                               hipStream_t stream) {
    if (n_tiles > 0)
        hipLaunchKernelGGL(k_batch_output, dim3(std::min<int32_t>(n_tiles, 8192)), dim3(kBlock), 0, stream, members,
                           tiles, n_tiles);
    if (n_members > 0)
        hipLaunchKernelGGL(k_batch_score, dim3(n_members), dim3(kBlock), 0, stream, members, member_ids, states_out);
    return hipGetLastError();
}

hipError_t launch_batch_states(const BatchMember *members, const int32_t *member_ids, int32_t n_members,
                               PrState *states_out, hipStream_t stream) {
    if (n_members > 0)
        hipLaunchKernelGGL(k_batch_states, dim3((n_members + 63) / 64), dim3(64), 0, stream, members, member_ids,
                           n_members, states_out);
    return hipGetLastError();
}

}  // namespace fl
