// fl_engine.hip - host side of the fitness-flow-graph engine: contexts, the
// device-memory cache, plans and the C ABI declared in include/fl.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "fl.h"
#include "fl_internal.h"

namespace {

using fl::BuildSizes;
using fl::PrArgs;
using fl::PrState;
using fl::SpaceDesc;

// Caching device allocator: buffers released by plans go to a free list keyed
// by their rounded size and are handed out again, so repeated analyses of
// similar spaces make no hipMalloc calls.  Sizes are rounded to a power of two
// up to 2 MiB and to whole 2 MiB pages above.
class DevicePool {
  public:
    ~DevicePool() { release_all(); }

    static size_t round_size(size_t n) {
        if (n == 0) n = 1;
        const size_t page = size_t(2) << 20;
        if (n <= page) {
            size_t p = 256;
            while (p < n) p <<= 1;
            return p;
        }
        return (n + page - 1) / page * page;
    }

    void *alloc(size_t bytes) {
        const size_t sz = round_size(bytes);
        auto it = free_.lower_bound(sz);
        if (it != free_.end() && it->first <= sz + sz / 2) {
            void *p = it->second;
            live_[p] = it->first;
            free_.erase(it);
            return p;
        }
        void *p = nullptr;
        if (hipMalloc(&p, sz) != hipSuccess) {
            (void)hipGetLastError();
            trim();
            if (hipMalloc(&p, sz) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
        }
        live_[p] = sz;
        return p;
    }

    void release(void *p) {
        if (!p) return;
        auto it = live_.find(p);
        if (it == live_.end()) return;
        free_.emplace(it->second, p);
        live_.erase(it);
    }

    void trim() {
        for (auto &kv : free_) (void)hipFree(kv.second);
        free_.clear();
    }

    void release_all() {
        trim();
        for (auto &kv : live_) (void)hipFree(kv.first);
        live_.clear();
    }

  private:
    std::multimap<size_t, void *> free_;
    std::map<void *, size_t> live_;
};

}  // namespace

struct fl_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cus = 256;
    std::string err;
    DevicePool pool;
    BuildSizes *h_sizes = nullptr;  // pinned
    PrState *h_state = nullptr;     // pinned
};

struct fl_plan {
    fl_ctx *ctx = nullptr;
    SpaceDesc sp{};
    int adjacent = 0;
    int64_t n_raw = 0, n = 0, e = 0, m = 0;
    float f_opt = 0.0f;
    // FFG, kept for fl_execute / fl_plan_export
    int32_t *valid_raw = nullptr;
    int32_t *out_deg = nullptr;
    int32_t *row_ptr = nullptr;
    int32_t *col_idx = nullptr;
    int32_t *minima = nullptr;
    float *fit_c = nullptr;
    uint64_t *rec = nullptr;    // node records (in-edge slot bits, out_deg, raw index)
    uint64_t *presence = nullptr;  // per wave of 64 nodes: OR of their slot bits
    fl::SlotTable sl{};
    // power-iteration working set, allocated by the first fl_execute
    float *y[2] = {nullptr, nullptr};
    float *x[2] = {nullptr, nullptr};
    int64_t x_cap = 0;          // entries of each x buffer
    double *partials = nullptr;
    PrState *state = nullptr;
    int pr_grid = 0;
    // timing
    hipEvent_t ev[7] = {};  // build 0-1, pagerank 2-3, score 4, iteration chunk 5-6
    bool have_events = false;
    fl_timing timing{};
};

namespace {

fl_status fail(fl_ctx *ctx, fl_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return st;
}

#define FL_HIP(call)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, FL_EHIP, "%s failed: %s", #call, hipGetErrorString(e_));       \
    } while (0)

template <typename T>
T *pool_alloc(fl_ctx *ctx, int64_t count) {
    return static_cast<T *>(ctx->pool.alloc(sizeof(T) * (size_t)std::max<int64_t>(count, 1)));
}

void release_plan_buffers(fl_plan *p) {
    DevicePool &pool = p->ctx->pool;
    void *bufs[] = {p->valid_raw, p->out_deg, p->row_ptr, p->col_idx, p->minima, p->fit_c, p->rec, p->presence,
                    p->y[0],      p->y[1],    p->x[0],    p->x[1],    p->partials, p->state};
    for (void *b : bufs) pool.release(b);
}

// Lanes per row for the iteration sweep: about half the mean in-degree, so a
// row's in-edges take two rounds of coalesced loads.
int auto_lanes(int64_t n, int64_t e) {
    const double mean = n > 0 ? (double)e / (double)n : 0.0;
    int l = 1;
    while (l < 64 && 2.0 * l < mean) l <<= 1;
    return l;
}

bool valid_lanes(int l) { return l == 1 || l == 2 || l == 4 || l == 8 || l == 16 || l == 32 || l == 64; }

// q / d == (q * m) >> (32 + l) for every q < 2^31, with l = ceil(log2 d) and
// m = ceil(2^(32+l) / d) < 2^34 (Granlund and Montgomery, "Division by
// invariant integers using multiplication", 1994, Thm. 4.2).
void set_magic(SpaceDesc &sp) {
    for (int k = 0; k < sp.n; ++k) {
        const uint64_t d = (uint64_t)sp.radix[k];
        uint32_t l = 0;
        while ((uint64_t(1) << l) < d) ++l;
        const uint32_t sh = 32 + l;
        const unsigned __int128 num = (unsigned __int128)1 << sh;
        sp.magic[k] = (uint64_t)((num + d - 1) / d);
        sp.shift[k] = sh;
    }
}

// Candidate slots sorted by raw-index offset: Hamming gives parameter k the
// deltas +-1 .. +-(radix_k - 1), adjacent +-1.  A node record holds the slot
// bits plus 40 bits of out_deg and raw index, in at most fl::kMaxWords words.
fl::SlotTable make_slots(const SpaceDesc &sp, bool adjacent) {
    fl::SlotTable t{};
    int64_t total = 0;
    for (int k = 0; k < sp.n; ++k) total += adjacent ? (sp.radix[k] > 1 ? 2 : 0) : 2 * ((int64_t)sp.radix[k] - 1);
    t.k = (int32_t)std::min<int64_t>(total, INT32_MAX);
    const int64_t words = (total + 40 + 63) / 64;
    if (total > fl::kMaxSlots || words > fl::kMaxWords) {
        t.words = 0;
        return t;
    }
    t.words = (int32_t)words;
    struct Slot { int64_t off; int delta, dim; };
    std::vector<Slot> slots;
    for (int k = 0; k < sp.n; ++k) {
        const int reach = adjacent ? std::min(1, sp.radix[k] - 1) : sp.radix[k] - 1;
        for (int dl = 1; dl <= reach; ++dl) {
            slots.push_back({-(int64_t)dl * sp.stride[k], -dl, k});
            slots.push_back({(int64_t)dl * sp.stride[k], dl, k});
        }
    }
    std::sort(slots.begin(), slots.end(), [](const Slot &x, const Slot &y) { return x.off < y.off; });
    for (size_t s = 0; s < slots.size(); ++s) {
        t.off[s] = (int32_t)slots[s].off;
        t.delta[s] = (int16_t)slots[s].delta;
        t.dim[s] = (uint8_t)slots[s].dim;
    }
    return t;
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return 0.0f;
    }
    return ms;
}

}  // namespace

extern "C" {

fl_status fl_create(fl_ctx **out, int device, void *hip_stream) {
    if (!out) return FL_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return FL_EINVAL;
    }
    fl_ctx *ctx = new (std::nothrow) fl_ctx;
    if (!ctx) return FL_ENOMEM;
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(device) != hipSuccess ||
        hipDeviceGetAttribute(&ctx->num_cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_sizes, sizeof(BuildSizes), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_state, sizeof(PrState), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        if (ctx->h_sizes) (void)hipHostFree(ctx->h_sizes);
        delete ctx;
        return FL_EHIP;
    }
    *out = ctx;
    return FL_OK;
}

fl_status fl_destroy(fl_ctx *ctx) {
    if (!ctx) return FL_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->pool.release_all();
    (void)hipHostFree(ctx->h_sizes);
    (void)hipHostFree(ctx->h_state);
    delete ctx;
    return FL_OK;
}

const char *fl_last_error(const fl_ctx *ctx) {
    if (!ctx) return "null context";
    return ctx->err.c_str();
}

fl_status fl_plan_create(fl_ctx *ctx, const fl_space *space, const float *d_fitness_raw,
                         fl_neighbourhood nb, fl_plan **out, fl_summary *sizes) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!out || !space || !d_fitness_raw) return fail(ctx, FL_EINVAL, "null argument");
    *out = nullptr;
    if (space->n_params < 1 || space->n_params > fl::kMaxParams || !space->radix)
        return fail(ctx, FL_EINVAL, "n_params must be in [1, %d]", fl::kMaxParams);
    if (nb != FL_NB_HAMMING && nb != FL_NB_ADJACENT)
        return fail(ctx, FL_EINVAL, "unknown neighbourhood %d", (int)nb);
    SpaceDesc sp{};
    sp.n = space->n_params;
    int64_t n_raw = 1;
    for (int i = 0; i < sp.n; ++i) {
        if (space->radix[i] < 1) return fail(ctx, FL_EINVAL, "radix[%d] = %d < 1", i, space->radix[i]);
        sp.radix[i] = space->radix[i];
        n_raw *= space->radix[i];
        if (n_raw >= (int64_t(1) << 31)) return fail(ctx, FL_EOVERFLOW, "prod radix >= 2^31");
    }
    for (int i = sp.n - 1; i >= 0; --i) sp.stride[i] = (i == sp.n - 1) ? 1 : sp.stride[i + 1] * sp.radix[i + 1];
    sp.n_raw = (int32_t)n_raw;
    set_magic(sp);
    FL_HIP(hipSetDevice(ctx->device));

    fl_plan *p = new (std::nothrow) fl_plan;
    if (!p) return fail(ctx, FL_ENOMEM, "out of host memory");
    p->ctx = ctx;
    p->sp = sp;
    p->adjacent = (nb == FL_NB_ADJACENT);
    p->sl = make_slots(sp, p->adjacent);
    p->n_raw = n_raw;
    for (auto &e : p->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            delete p;
            return fail(ctx, FL_EHIP, "hipEventCreate failed");
        }
    }
    p->have_events = true;
    hipStream_t s = ctx->stream;

    // scratch that lives only during the build
    const int64_t c_tiles = (n_raw + fl::kCompactTile - 1) / fl::kCompactTile;
    int32_t *remap = pool_alloc<int32_t>(ctx, n_raw);
    int32_t *tile_cnt = pool_alloc<int32_t>(ctx, c_tiles);
    int32_t *tile_bad = pool_alloc<int32_t>(ctx, c_tiles);
    int32_t *tile_off = pool_alloc<int32_t>(ctx, c_tiles);
    float *tile_min = pool_alloc<float>(ctx, c_tiles);
    BuildSizes *d_sizes = pool_alloc<BuildSizes>(ctx, 1);
    p->valid_raw = pool_alloc<int32_t>(ctx, n_raw);
    p->fit_c = pool_alloc<float>(ctx, n_raw);
    std::vector<void *> scratch = {remap, tile_cnt, tile_bad, tile_off, tile_min, d_sizes};
    auto cleanup = [&](fl_status st) {
        (void)hipStreamSynchronize(s);
        for (void *b : scratch) ctx->pool.release(b);
        if (st != FL_OK) {
            release_plan_buffers(p);
            for (auto &e : p->ev) (void)hipEventDestroy(e);
            delete p;
        }
        return st;
    };
    for (void *b : scratch)
        if (!b) return cleanup(fail(ctx, FL_ENOMEM, "device allocation failed"));
    if (!p->valid_raw || !p->fit_c) return cleanup(fail(ctx, FL_ENOMEM, "device allocation failed"));

    hipError_t he = hipEventRecord(p->ev[0], s);
    if (he == hipSuccess)
        he = fl::launch_compact(d_fitness_raw, sp.n_raw, tile_cnt, tile_min, tile_bad, tile_off, remap,
                                p->valid_raw, p->fit_c, d_sizes, s);
    if (he == hipSuccess) he = hipMemcpyAsync(ctx->h_sizes, d_sizes, sizeof(BuildSizes), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return cleanup(fail(ctx, FL_EHIP, "compaction: %s", hipGetErrorString(he)));
    if (ctx->h_sizes->n_bad > 0)
        return cleanup(fail(ctx, FL_EINVAL, "%d fitness values are <= 0 or -inf", ctx->h_sizes->n_bad));
    const int32_t n = ctx->h_sizes->n_valid;
    if (n == 0) return cleanup(fail(ctx, FL_EINVAL, "no valid configuration (all NaN / +inf)"));
    p->n = n;
    p->f_opt = ctx->h_sizes->f_opt;

    const int64_t n_tiles = (n + fl::kBlock - 1) / fl::kBlock;
    int32_t *in_deg = pool_alloc<int32_t>(ctx, n);
    int64_t *tile_e = pool_alloc<int64_t>(ctx, n_tiles);
    int64_t *tile_eoff = pool_alloc<int64_t>(ctx, n_tiles);
    int32_t *tile_m = pool_alloc<int32_t>(ctx, n_tiles);
    int32_t *tile_moff = pool_alloc<int32_t>(ctx, n_tiles);
    scratch.insert(scratch.end(), {in_deg, tile_e, tile_eoff, tile_m, tile_moff});
    p->out_deg = pool_alloc<int32_t>(ctx, n);
    p->row_ptr = pool_alloc<int32_t>(ctx, (int64_t)n + 1);
    p->minima = pool_alloc<int32_t>(ctx, n);
    if (p->sl.words > 0) {
        p->rec = pool_alloc<uint64_t>(ctx, (int64_t)n * p->sl.words);
        p->presence = pool_alloc<uint64_t>(ctx, ((int64_t)n + 63) / 64 * p->sl.words);
    }
    for (void *b : scratch)
        if (!b) return cleanup(fail(ctx, FL_ENOMEM, "device allocation failed"));
    if (!p->out_deg || !p->row_ptr || !p->minima || (p->sl.words > 0 && (!p->rec || !p->presence)))
        return cleanup(fail(ctx, FL_ENOMEM, "device allocation failed"));

    he = fl::launch_degree(sp, p->sl, p->adjacent, d_fitness_raw, p->valid_raw, n, in_deg, p->out_deg, p->rec,
                           p->presence, tile_e, tile_m, tile_eoff, tile_moff, d_sizes, s);
    if (he == hipSuccess) he = hipMemcpyAsync(ctx->h_sizes, d_sizes, sizeof(BuildSizes), hipMemcpyDeviceToHost, s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return cleanup(fail(ctx, FL_EHIP, "degree count: %s", hipGetErrorString(he)));
    const int64_t e = ctx->h_sizes->n_edges;
    if (e >= (int64_t(1) << 31)) return cleanup(fail(ctx, FL_EOVERFLOW, "edge count %lld >= 2^31", (long long)e));
    p->e = e;
    p->m = ctx->h_sizes->n_minima;
    p->col_idx = pool_alloc<int32_t>(ctx, e);
    if (!p->col_idx) return cleanup(fail(ctx, FL_ENOMEM, "device allocation failed"));

    he = fl::launch_fill(sp, p->sl, p->adjacent, d_fitness_raw, p->valid_raw, remap, p->rec, n, (int32_t)e,
                         in_deg, p->out_deg, tile_eoff, tile_moff, p->row_ptr, p->col_idx, p->minima, s);
    if (he == hipSuccess) he = hipEventRecord(p->ev[1], s);
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (he != hipSuccess) return cleanup(fail(ctx, FL_EHIP, "CSR fill: %s", hipGetErrorString(he)));
    p->timing.build_ms = elapsed(p->ev[0], p->ev[1]);

    if (sizes) {
        memset(sizes, 0, sizeof *sizes);
        sizes->n_raw = p->n_raw;
        sizes->n_valid = p->n;
        sizes->n_edges = p->e;
        sizes->n_minima = p->m;
        sizes->n_slots = p->sl.k;
        sizes->mask_words = p->sl.words;
        sizes->f_opt = (double)p->f_opt;
    }
    *out = p;
    return cleanup(FL_OK);
}

fl_status fl_execute(fl_ctx *ctx, fl_plan *p, const fl_params *prm, double *d_pagerank,
                     int32_t *d_minima, fl_summary *out) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!p || !prm || !d_pagerank || (!d_minima && p->m > 0)) return fail(ctx, FL_EINVAL, "null argument");
    if (p->ctx != ctx) return fail(ctx, FL_EINVAL, "plan belongs to another context");
    const double d = prm->damping;
    if (!(d > 0.0 && d < 1.0)) return fail(ctx, FL_EINVAL, "damping must be in (0,1)");
    if (!(prm->p >= 0.0) || !isfinite(prm->p)) return fail(ctx, FL_EINVAL, "p must be finite and >= 0");
    if (!(prm->tol_l1 >= 0.0) || !isfinite(prm->tol_l1)) return fail(ctx, FL_EINVAL, "tol_l1 must be finite and >= 0");
    if (prm->max_iter < 0) return fail(ctx, FL_EINVAL, "max_iter must be >= 0");
    if (prm->row_mapping != 0 && prm->row_mapping != FL_ROWS_SLOTS && !valid_lanes(prm->row_mapping))
        return fail(ctx, FL_EINVAL, "row_mapping must be 0, FL_ROWS_SLOTS or a power of two <= 64");
    if (prm->row_mapping == FL_ROWS_SLOTS && p->sl.words == 0)
        return fail(ctx, FL_EINVAL, "the slot sweep needs at most %d candidate slots (space has %d)",
                    fl::kMaxSlots, p->sl.k);
    const double tol = prm->tol_l1 > 0.0 ? prm->tol_l1 : 2e-7;
    const int32_t max_iter = prm->max_iter > 0 ? prm->max_iter : 1000;
    int lanes = prm->row_mapping;
    if (lanes == 0) lanes = p->sl.words > 0 ? FL_ROWS_SLOTS : auto_lanes(p->n, p->e);
    const int kind = lanes == FL_ROWS_SLOTS ? fl::kSweepSlots : fl::kSweepCsr;
    FL_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;

    PrArgs a{};
    a.kind = kind;
    a.adjacent = p->adjacent;
    // persistent grid: every workgroup resident at once (occupancy query), a
    // multiple of the XCD count so each XCD gets the same number of them
    int per_cu = 0;
    FL_HIP(fl::pr_iter_blocks_per_cu(a, p->sp, p->sl, lanes, &per_cu));
    const int64_t resident = std::max<int64_t>(fl::kXcds, (int64_t)std::max(per_cu, 1) * ctx->num_cus / fl::kXcds * fl::kXcds);
    const int64_t rows_per_wg = kind == fl::kSweepSlots ? fl::kBlock : fl::kBlock / lanes;
    const int64_t groups = (p->n + rows_per_wg - 1) / rows_per_wg;
    const int grid = (int)std::min<int64_t>(resident, (groups + fl::kXcds - 1) / fl::kXcds * fl::kXcds);
    const int64_t x_need = kind == fl::kSweepSlots ? p->n_raw : p->n;
    if (!p->state) {
        for (int j = 0; j < 2; ++j) p->y[j] = pool_alloc<float>(ctx, p->n);
        p->state = pool_alloc<PrState>(ctx, 1);
        if (!p->y[0] || !p->y[1] || !p->state) return fail(ctx, FL_ENOMEM, "device allocation failed");
    }
    if (x_need > p->x_cap) {
        for (int j = 0; j < 2; ++j) {
            ctx->pool.release(p->x[j]);
            p->x[j] = pool_alloc<float>(ctx, x_need);
        }
        if (!p->x[0] || !p->x[1]) return fail(ctx, FL_ENOMEM, "device allocation failed");
        p->x_cap = x_need;
    }
    // the init and iteration kernels each write 3 partial sums per workgroup
    const int init_grid = (int)std::min<int64_t>((p->n + fl::kBlock - 1) / fl::kBlock, (int64_t)ctx->num_cus * 4);
    const int need = std::max(grid, init_grid);
    if (need > p->pr_grid) {
        ctx->pool.release(p->partials);
        p->partials = pool_alloc<double>(ctx, 3 * (int64_t)need);
        if (!p->partials) return fail(ctx, FL_ENOMEM, "device allocation failed");
        p->pr_grid = need;
    }
    a.row_ptr = p->row_ptr;
    a.col_idx = p->col_idx;
    a.out_deg = p->out_deg;
    a.valid_raw = p->valid_raw;
    a.rec = p->rec;
    a.presence = p->presence;
    a.x_bytes = (kind == fl::kSweepSlots && 4 * p->n_raw < (int64_t(1) << 31)) ? (int32_t)(4 * p->n_raw) : 0;
    a.y[0] = p->y[0];
    a.y[1] = p->y[1];
    a.x[0] = p->x[0];
    a.x[1] = p->x[1];
    a.partials = p->partials;
    a.st = p->state;
    a.n = (int32_t)p->n;
    a.d = d;
    a.tol = tol;
    a.max_iter = max_iter;

    FL_HIP(hipEventRecord(p->ev[2], s));
    FL_HIP(hipMemsetAsync(p->state, 0, sizeof(PrState), s));
    FL_HIP(fl::launch_pr_init(a, init_grid, s));

    // Launch the iteration kernel in chunks; a launch after convergence exits
    // at once.  The chunk length follows the observed residual decay so that
    // few host round trips and few empty launches are needed.
    int launches = 0;
    int chunk = 16;
    double iterate_ms = 0.0;
    PrState *hs = ctx->h_state;
    for (;;) {
        FL_HIP(hipEventRecord(p->ev[5], s));
        for (int j = 0; j < chunk; ++j) FL_HIP(fl::launch_pr_iter(a, p->sp, p->sl, lanes, grid, s));
        FL_HIP(hipEventRecord(p->ev[6], s));
        launches += chunk;
        FL_HIP(hipMemcpyAsync(hs, p->state, sizeof(PrState), hipMemcpyDeviceToHost, s));
        FL_HIP(hipStreamSynchronize(s));
        iterate_ms += elapsed(p->ev[5], p->ev[6]);
        if (hs->done) break;
        const double rate = (hs->resid_prev > 0.0) ? hs->resid / hs->resid_prev : 1.0;
        if (rate > 0.0 && rate < 0.999 && hs->resid > tol) {
            const double more = ceil(log(tol / hs->resid) / log(rate));
            chunk = (int)std::min(64.0, std::max(2.0, more + 1.0));
        } else {
            chunk = 8;
        }
        chunk = std::min(chunk, std::max(1, max_iter - hs->k));
    }
    FL_HIP(hipEventRecord(p->ev[3], s));
    FL_HIP(fl::launch_pr_output(a, d_pagerank, s));
    if (p->m > 0) FL_HIP(hipMemcpyAsync(d_minima, p->minima, sizeof(int32_t) * p->m, hipMemcpyDeviceToDevice, s));
    const double threshold = (1.0 + prm->p) * (double)p->f_opt;
    FL_HIP(fl::launch_score(d_pagerank, p->minima, (int32_t)p->m, p->fit_c, threshold, p->state, s));
    FL_HIP(hipEventRecord(p->ev[4], s));
    FL_HIP(hipMemcpyAsync(hs, p->state, sizeof(PrState), hipMemcpyDeviceToHost, s));
    FL_HIP(hipStreamSynchronize(s));

    p->timing.pagerank_ms = elapsed(p->ev[2], p->ev[3]);
    p->timing.score_ms = elapsed(p->ev[3], p->ev[4]);
    p->timing.iterate_ms = iterate_ms;
    p->timing.iterations = hs->worked;
    p->timing.launches = launches;
    if (out) {
        memset(out, 0, sizeof *out);
        out->n_raw = p->n_raw;
        out->n_valid = p->n;
        out->n_edges = p->e;
        out->n_minima = p->m;
        out->iterations = hs->k;
        out->row_mapping = lanes;
        out->n_slots = p->sl.k;
        out->mask_words = p->sl.words;
        out->residual_l1 = hs->resid;
        out->f_opt = (double)p->f_opt;
        out->mass_minima = hs->score_den;
        out->mass_near = hs->score_num;
        out->score = hs->score_den > 0.0 ? hs->score_num / hs->score_den : 0.0;
    }
    if (hs->done != 1)
        return fail(ctx, FL_ENOCONV, "no convergence after %d iterations (residual %.3e)", hs->k, hs->resid);
    return FL_OK;
}

fl_status fl_plan_export(fl_ctx *ctx, const fl_plan *p, int32_t *d_valid_raw, int32_t *d_row_ptr,
                         int32_t *d_col_idx, int32_t *d_out_deg) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!p || p->ctx != ctx) return fail(ctx, FL_EINVAL, "bad plan");
    FL_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    if (d_valid_raw) FL_HIP(hipMemcpyAsync(d_valid_raw, p->valid_raw, 4 * p->n, hipMemcpyDeviceToDevice, s));
    if (d_row_ptr) FL_HIP(hipMemcpyAsync(d_row_ptr, p->row_ptr, 4 * (p->n + 1), hipMemcpyDeviceToDevice, s));
    if (d_col_idx && p->e > 0) FL_HIP(hipMemcpyAsync(d_col_idx, p->col_idx, 4 * p->e, hipMemcpyDeviceToDevice, s));
    if (d_out_deg) FL_HIP(hipMemcpyAsync(d_out_deg, p->out_deg, 4 * p->n, hipMemcpyDeviceToDevice, s));
    return FL_OK;
}

fl_status fl_plan_timing(fl_ctx *ctx, const fl_plan *p, fl_timing *out) {
    if (!ctx) return FL_EINVAL;
    if (!p || !out || p->ctx != ctx) return fail(ctx, FL_EINVAL, "bad argument");
    *out = p->timing;
    return FL_OK;
}

fl_status fl_plan_destroy(fl_ctx *ctx, fl_plan *p) {
    if (!ctx) return FL_EINVAL;
    if (!p) return FL_OK;
    if (p->ctx != ctx) return fail(ctx, FL_EINVAL, "plan belongs to another context");
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    release_plan_buffers(p);
    if (p->have_events)
        for (auto &e : p->ev) (void)hipEventDestroy(e);
    delete p;
    return FL_OK;
}

fl_status fl_analyze(fl_ctx *ctx, const fl_space *space, const float *d_fitness_raw, fl_neighbourhood nb,
                     const fl_params *params, double *d_pagerank, int32_t *d_minima, int32_t *d_valid_raw,
                     fl_summary *out) {
    if (!ctx) return FL_EINVAL;
    fl_plan *p = nullptr;
    fl_status st = fl_plan_create(ctx, space, d_fitness_raw, nb, &p, nullptr);
    if (st != FL_OK) return st;
    st = fl_execute(ctx, p, params, d_pagerank, d_minima, out);
    if (st == FL_OK || st == FL_ENOCONV) {
        const fl_status xs = fl_plan_export(ctx, p, d_valid_raw, nullptr, nullptr, nullptr);
        if (xs != FL_OK) st = xs;
    }
    const std::string msg = ctx->err;
    fl_plan_destroy(ctx, p);
    ctx->err = msg;
    return st;
}

}  // extern "C"
