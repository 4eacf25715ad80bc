// fl_engine.hip - host side of the fitness-flow-graph engine: contexts, the
// device-memory cache, plans and the C ABI declared in include/fl.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
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

// Bump allocator over the scratch array of fl_analyze_noalloc: while a
// context has one installed, every device buffer of a build and an execute
// is carved from it in 256-byte aligned pieces, and nothing is freed.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    bool overflow = false;

    void *take(size_t bytes) {
        const size_t need = (bytes + 255) / 256 * 256;
        if (overflow || need > cap - used) {
            overflow = true;
            return nullptr;
        }
        void *p = base + used;
        used += need;
        return p;
    }
};

}  // namespace

// Scratch memory of fl_analyze_noalloc (callers that cannot allocate device
// memory): one array on every device the library runs on, held until the
// process ends.  Host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (scratch_address).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxScratchDevices] = {};

// Device address of `scratch` on `device` (which must be current), looked up
// once per device.
hipError_t scratch_address(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = ptr;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

}  // namespace

struct fl_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cus = 256;
    std::string err;
    DevicePool pool;
    std::map<uint64_t, int> tuned;  // shape class -> sweep layout chosen by fl_tune
    std::map<uint64_t, uint64_t> tuned_map;  // shape class -> in-degree bucket mapping chosen by fl_tune
    int32_t *h_bins = nullptr;      // pinned: bucket classes out, class sizes back
    int32_t profile_every = 0;      // bracket every n-th sweep kernel with events (fl_profile), 0 = off
    std::vector<hipEvent_t> sweep_ev;  // 2 per launch of the longest chunk so far
    BuildSizes *h_sizes = nullptr;  // pinned
    PrState *h_state = nullptr;     // pinned
    fl_batch *analyze_batch = nullptr;  // kept by fl_analyze_batch between calls (empty between calls)
    // pinned tables of the segmented build (fl_analyze_batch), grown on demand
    fl::SegBuild *h_segs = nullptr;
    BuildSizes *h_seg_sizes = nullptr;  // the spaces' sizes, copied back once per stage
    fl::SegTile *h_seg_tiles = nullptr;
    int32_t *h_seg_ids = nullptr;
    int32_t seg_cap = 0;
    int64_t seg_tile_cap = 0;
    void *scratch = nullptr;  // this device's address of the no-allocation scratch array
    Arena *arena = nullptr;   // installed by fl_analyze_noalloc for the length of the call
};

struct fl_plan {
    fl_ctx *ctx = nullptr;
    SpaceDesc sp{};
    int adjacent = 0;
    int64_t n_raw = 0, n = 0, e = 0, m = 0;
    int32_t n_plateau = 0;
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
    float *y[3] = {nullptr, nullptr, nullptr};   // the third for the lagged step
    float *x[2] = {nullptr, nullptr};
    float *g = nullptr;         // lagged step: the first sweep's edge sums (node ids)
    int64_t x_cap = 0;          // entries of each x buffer
    double *partials = nullptr;
    PrState *state = nullptr;
    int pr_grid = 0;
    // rows binned by in-degree (binned sweep): node ids grouped by class,
    // the classes, and the bucket mapping they were built for
    int32_t *bin_rows = nullptr;
    fl::BinTable bins{};
    uint64_t bin_map = 0;
    bool have_bins = false;
    int32_t bin_users = 0;      // batch members sweeping these bins (no rebinning meanwhile)
    int32_t *d_off = nullptr;   // 2 k_pad entries in device memory, read by the slot sweep:
                                // raw-index offsets, then byte offsets from the most negative
                                // (written by the degree kernel)
    // timing
    hipEvent_t ev[7] = {};  // build 0-1, pagerank 2-3, score 4, iteration chunk 5-6
    bool have_events = false;   // created on first use (plans of fl_analyze_batch never time)
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

// Device buffer of `count` T from the context's pool, or from the scratch
// arena while fl_analyze_noalloc runs (pool.release ignores arena pieces).
template <typename T>
T *pool_alloc(fl_ctx *ctx, int64_t count) {
    const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    if (ctx->arena) return static_cast<T *>(ctx->arena->take(bytes));
    return static_cast<T *>(ctx->pool.alloc(bytes));
}

// Several device buffers carved from one pool block in 256-byte aligned
// pieces, so that a build stage or a batch member costs one pool operation
// (a batched build of a few hundred spaces made thousands, about 0.1 us of
// host time each).  The first piece is the block's base: releasing it
// returns the block, and the pool ignores the other pieces' pointers.
class Carve {
  public:
    template <typename T>
    Carve &add(T *&dst, int64_t count) {
        if (n_ < kMax) piece_[n_++] = {reinterpret_cast<void **>(&dst), sizeof(T) * (size_t)std::max<int64_t>(count, 1)};
        else overflow_ = true;
        return *this;
    }
    // false (every destination null) when the block cannot be had
    bool take(fl_ctx *ctx) {
        size_t total = 0;
        for (int j = 0; j < n_; ++j) total += round(piece_[j].bytes);
        char *base = overflow_ ? nullptr : pool_alloc<char>(ctx, (int64_t)total);
        size_t off = 0;
        for (int j = 0; j < n_; ++j) {
            *piece_[j].dst = base ? base + off : nullptr;
            off += round(piece_[j].bytes);
        }
        return base != nullptr;
    }

  private:
    static size_t round(size_t b) { return (b + 255) / 256 * 256; }
    static constexpr int kMax = 8;
    struct Piece {
        void **dst;
        size_t bytes;
    };
    Piece piece_[kMax] = {};
    int n_ = 0;
    bool overflow_ = false;
};

void release_plan_buffers(fl_plan *p) {
    DevicePool &pool = p->ctx->pool;
    void *bufs[] = {p->valid_raw, p->out_deg, p->row_ptr, p->col_idx, p->minima,  p->fit_c,
                    p->rec,       p->presence, p->y[0], p->y[1],      p->y[2],     p->x[0],
                    p->x[1],      p->g,       p->partials, p->state,  p->d_off,    p->bin_rows};
    for (void *b : bufs) pool.release(b);
}

// A plan's buffers back to the pool and its events destroyed; the caller has
// synchronised the stream that last used them.
void plan_free(fl_plan *p) {
    release_plan_buffers(p);
    if (p->have_events)
        for (auto &e : p->ev) (void)hipEventDestroy(e);
    delete p;
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
// Stride of the two halves of the device offset table: the sweep reads whole
// batches of offsets (up to 64 past the last slot), so k rounded up to 64, plus 64.
int32_t k_pad_of(const fl::SlotTable &sl) { return (sl.k + 63) / 64 * 64 + 64; }

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
    Slot slots[fl::kMaxSlots];
    int n_slots = 0;
    for (int k = 0; k < sp.n; ++k) {
        const int reach = adjacent ? std::min(1, sp.radix[k] - 1) : sp.radix[k] - 1;
        for (int dl = 1; dl <= reach; ++dl) {
            slots[n_slots++] = {-(int64_t)dl * sp.stride[k], -dl, k};
            slots[n_slots++] = {(int64_t)dl * sp.stride[k], dl, k};
        }
    }
    std::sort(slots, slots + n_slots, [](const Slot &x, const Slot &y) { return x.off < y.off; });
    for (int s = 0; s < n_slots; ++s) {
        t.off[s] = (int32_t)slots[s].off;
        t.delta[s] = (int16_t)slots[s].delta;
        t.dim[s] = (uint8_t)slots[s].dim;
    }
    // runs of each parameter's slots (checked: a space where they were not
    // contiguous would take the generic kernels)
    for (int k = 0; k < sp.n; ++k) {
        const int reach = adjacent ? std::min(1, sp.radix[k] - 1) : sp.radix[k] - 1;
        t.blk_len[k] = (int16_t)reach;
        t.blk_neg[k] = t.blk_pos[k] = 0;
        if (reach <= 0) continue;
        int neg = -1, pos = -1;
        for (int s = 0; s < t.k; ++s) {
            if (t.dim[s] != k) continue;
            if (t.delta[s] == -reach) neg = s;
            if (t.delta[s] == 1) pos = s;
        }
        bool ok = neg >= 0 && pos >= 0;
        for (int d = 0; ok && d < reach; ++d)
            ok = t.dim[neg + d] == k && t.delta[neg + d] == d - reach && t.dim[pos + d] == k && t.delta[pos + d] == d + 1;
        if (!ok) {
            t.words = 0;
            return t;
        }
        t.blk_neg[k] = (int16_t)neg;
        t.blk_pos[k] = (int16_t)pos;
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


// ---------------------------------------------------------------------------
// Plan building in resumable stages, so that many spaces can be built with one
// host synchronisation per stage (fl_analyze_batch) as well as one at a time.

struct Build {
    fl_plan *p = nullptr;
    fl_status status = FL_OK;
    std::string err;
    bool timed = true;              // record build events (fl_plan_create)
    bool shared_sizes = false;      // d_sizes is a slot of a caller-owned array that the
                                    // caller copies to h_sizes itself (fl_analyze_batch)
    bool defer = false;             // allocate only: the caller launches the stage's kernels for
                                    // many builds at once (segmented build; slot spaces and
                                    // compaction only, the generic kernels still launch here)
    BuildSizes *h_sizes = nullptr;  // pinned slot for this build's sizes
    fl_plan *storage = nullptr;     // caller-owned plan object to build into (else one is allocated)
    const float *fit = nullptr;
    int32_t *remap = nullptr, *tile_cnt = nullptr, *tile_bad = nullptr, *tile_off = nullptr;
    float *tile_min = nullptr;
    BuildSizes *d_sizes = nullptr;
    int32_t *in_deg = nullptr, *tile_m = nullptr, *tile_moff = nullptr;
    int64_t *tile_e = nullptr, *tile_eoff = nullptr;
};

void build_fail(Build &b, fl_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    b.status = st;
    b.err = buf;
}

void build_release_scratch(fl_ctx *ctx, Build &b) {
    void *bufs[] = {b.remap, b.tile_cnt, b.tile_bad, b.tile_off, b.tile_min, b.shared_sizes ? nullptr : b.d_sizes,
                    b.in_deg, b.tile_m, b.tile_moff, b.tile_e, b.tile_eoff};
    for (void *x : bufs) ctx->pool.release(x);
    b.remap = b.tile_cnt = b.tile_bad = b.tile_off = b.in_deg = b.tile_m = b.tile_moff = nullptr;
    b.tile_min = nullptr;
    b.d_sizes = nullptr;
    b.tile_e = b.tile_eoff = nullptr;
}

// The plan's timing events, created on first use.
hipError_t ensure_events(fl_plan *p) {
    if (p->have_events) return hipSuccess;
    for (int j = 0; j < 7; ++j) {
        const hipError_t e = hipEventCreate(&p->ev[j]);
        if (e != hipSuccess) {
            for (int q = 0; q < j; ++q) (void)hipEventDestroy(p->ev[q]);
            return e;
        }
    }
    p->have_events = true;
    return hipSuccess;
}

void build_abort(fl_ctx *ctx, Build &b) {
    build_release_scratch(ctx, b);
    if (b.p) {
        release_plan_buffers(b.p);
        if (b.p->have_events)
            for (auto &e : b.p->ev) (void)hipEventDestroy(e);
        if (b.p != b.storage) delete b.p;
        b.p = nullptr;
    }
}

// Stage 1: validate, allocate, launch the compaction (Sec. III-B, Sec. V).
void build_begin(fl_ctx *ctx, Build &b, const fl_space *space, const float *fit, fl_neighbourhood nb) {
    if (!space || !fit) return build_fail(b, FL_EINVAL, "null argument");
    if (space->n_params < 1 || space->n_params > fl::kMaxParams || !space->radix)
        return build_fail(b, FL_EINVAL, "n_params must be in [1, %d]", fl::kMaxParams);
    if (nb != FL_NB_HAMMING && nb != FL_NB_ADJACENT)
        return build_fail(b, FL_EINVAL, "unknown neighbourhood %d", (int)nb);
    SpaceDesc sp{};
    sp.n = space->n_params;
    int64_t n_raw = 1;
    for (int i = 0; i < sp.n; ++i) {
        if (space->radix[i] < 1) return build_fail(b, FL_EINVAL, "radix[%d] = %d < 1", i, space->radix[i]);
        sp.radix[i] = space->radix[i];
        n_raw *= space->radix[i];
        if (n_raw >= (int64_t(1) << 31)) return build_fail(b, FL_EOVERFLOW, "prod radix >= 2^31");
    }
    for (int i = sp.n - 1; i >= 0; --i) sp.stride[i] = (i == sp.n - 1) ? 1 : sp.stride[i + 1] * sp.radix[i + 1];
    sp.n_raw = (int32_t)n_raw;
    set_magic(sp);

    fl_plan *p = b.storage;
    if (p) *p = fl_plan{};
    else p = new (std::nothrow) fl_plan;
    if (!p) return build_fail(b, FL_ENOMEM, "out of host memory");
    b.p = p;
    b.fit = fit;
    p->ctx = ctx;
    p->sp = sp;
    p->adjacent = (nb == FL_NB_ADJACENT);
    p->sl = make_slots(sp, p->adjacent);
    p->n_raw = n_raw;
    if (b.timed && ensure_events(p) != hipSuccess) {
        (void)hipGetLastError();
        return build_fail(b, FL_EHIP, "hipEventCreate failed");
    }

    // tiles of the segmented build's three passes, or of one space's two
    const int64_t c_tiles = b.defer ? (n_raw + fl::kCompactTile - 1) / fl::kCompactTile
                                    : (n_raw + fl::kSingleTile - 1) / fl::kSingleTile;
    // scratch (based at remap) and plan buffers (based at valid_raw), one block each
    Carve scratch;
    scratch.add(b.remap, n_raw).add(b.tile_cnt, c_tiles).add(b.tile_bad, c_tiles).add(b.tile_min, c_tiles);
    if (b.defer) scratch.add(b.tile_off, c_tiles);
    if (!b.shared_sizes) scratch.add(b.d_sizes, 1);
    scratch.take(ctx);
    Carve own;
    own.add(p->valid_raw, n_raw).add(p->fit_c, n_raw).take(ctx);
    if (!b.remap || !b.tile_cnt || !b.tile_bad || (b.defer && !b.tile_off) || !b.tile_min || !b.d_sizes ||
        !p->valid_raw || !p->fit_c)
        return build_fail(b, FL_ENOMEM, "device allocation failed");
    hipStream_t s = ctx->stream;
    hipError_t he = b.timed ? hipEventRecord(p->ev[0], s) : hipSuccess;
    if (he == hipSuccess && !b.defer)
        he = fl::launch_compact_single(fit, sp.n_raw, b.tile_cnt, b.tile_min, b.tile_bad, b.remap, p->valid_raw,
                                       p->fit_c, b.d_sizes, s);
    if (he == hipSuccess && !b.shared_sizes)
        he = hipMemcpyAsync(b.h_sizes, b.d_sizes, sizeof(BuildSizes), hipMemcpyDeviceToHost, s);
    if (he != hipSuccess) build_fail(b, FL_EHIP, "compaction: %s", hipGetErrorString(he));
}

// Stage 2 (sizes of stage 1 on the host): degree count + scans (Sec. VII-B).
void build_degree(fl_ctx *ctx, Build &b) {
    if (b.status != FL_OK) return;
    fl_plan *p = b.p;
    if (b.h_sizes->n_bad > 0)
        return build_fail(b, FL_EINVAL, "%d fitness values are <= 0 or -inf", b.h_sizes->n_bad);
    const int32_t n = b.h_sizes->n_valid;
    if (n == 0) return build_fail(b, FL_EINVAL, "no valid configuration (all NaN / +inf)");
    p->n = n;
    p->f_opt = b.h_sizes->f_opt;
    const int64_t n_tiles = (n + fl::kBlock - 1) / fl::kBlock;
    // scratch (based at in_deg) and plan buffers (based at out_deg), one block each
    Carve scratch;
    scratch.add(b.in_deg, n).add(b.tile_e, n_tiles).add(b.tile_eoff, n_tiles).add(b.tile_m, n_tiles);
    scratch.add(b.tile_moff, n_tiles).take(ctx);
    Carve own;
    own.add(p->out_deg, n).add(p->row_ptr, (int64_t)n + 1).add(p->minima, n);
    if (p->sl.words > 0) {
        own.add(p->rec, (int64_t)n * p->sl.words).add(p->presence, ((int64_t)n + 63) / 64 * p->sl.words);
        own.add(p->d_off, 2 * k_pad_of(p->sl));
    }
    own.take(ctx);
    if (!b.in_deg || !b.tile_e || !b.tile_eoff || !b.tile_m || !b.tile_moff || !p->out_deg || !p->row_ptr ||
        !p->minima || (p->sl.words > 0 && (!p->rec || !p->presence || !p->d_off)))
        return build_fail(b, FL_ENOMEM, "device allocation failed");
    hipStream_t s = ctx->stream;
    if (b.defer && p->sl.words > 0) return;
    hipError_t he = fl::launch_degree(p->sp, p->sl, p->adjacent, b.fit, p->valid_raw, n, b.in_deg, p->out_deg,
                                      p->rec, p->presence, p->d_off, k_pad_of(p->sl), b.tile_e, b.tile_m,
                                      b.tile_eoff, b.tile_moff, b.d_sizes, s);
    if (he == hipSuccess && !b.shared_sizes)
        he = hipMemcpyAsync(b.h_sizes, b.d_sizes, sizeof(BuildSizes), hipMemcpyDeviceToHost, s);
    if (he != hipSuccess) build_fail(b, FL_EHIP, "degree count: %s", hipGetErrorString(he));
}

// Stage 3 (edge count on the host): CSR fill and minima (Sec. III-B, VII-B).
void build_fill(fl_ctx *ctx, Build &b) {
    if (b.status != FL_OK) return;
    fl_plan *p = b.p;
    const int64_t e = b.h_sizes->n_edges;
    if (e >= (int64_t(1) << 31)) return build_fail(b, FL_EOVERFLOW, "edge count %lld >= 2^31", (long long)e);
    p->e = e;
    p->m = b.h_sizes->n_minima;
    p->n_plateau = b.h_sizes->n_plateau;
    p->col_idx = pool_alloc<int32_t>(ctx, e);
    if (!p->col_idx) return build_fail(b, FL_ENOMEM, "device allocation failed");
    hipStream_t s = ctx->stream;
    if (b.defer && p->sl.words > 0) return;
    hipError_t he = fl::launch_fill(p->sp, p->sl, p->adjacent, b.fit, p->valid_raw, b.remap, p->rec, p->presence,
                                    (int32_t)p->n, (int32_t)e, b.in_deg, p->out_deg, b.tile_eoff, b.tile_moff,
                                    p->row_ptr, p->col_idx, p->minima, s);
    if (he == hipSuccess && b.timed) he = hipEventRecord(p->ev[1], s);
    if (he != hipSuccess) build_fail(b, FL_EHIP, "CSR fill: %s", hipGetErrorString(he));
}

// Stage 4 (after the stream has drained): release scratch, record timing.
void build_end(fl_ctx *ctx, Build &b) {
    build_release_scratch(ctx, b);
    if (b.status != FL_OK || !b.timed) return;
    b.p->timing.build_ms = elapsed(b.p->ev[0], b.p->ev[1]);
}

void fill_sizes(const fl_plan *p, fl_summary *sizes) {
    memset(sizes, 0, sizeof *sizes);
    sizes->n_raw = p->n_raw;
    sizes->n_valid = p->n;
    sizes->n_edges = p->e;
    sizes->n_minima = p->m;
    sizes->n_plateau = p->n_plateau;
    sizes->n_slots = p->sl.k;
    sizes->mask_words = p->sl.words;
    sizes->f_opt = (double)p->f_opt;
}

// Analysis parameters with the defaults applied.
// Bytes the slot sweep's buffer loads span: its descriptor starts at the most
// negative slot offset below x, and the loads reach the end of x plus the
// largest offset; 0 when that does not fit a signed 32-bit offset (the
// sweep then uses plain loads).
int32_t x_bytes_of(const fl_plan *p) {
    if (p->sl.k <= 0) return 0;
    const int64_t span = (p->n_raw + 3) / 4 * 4 + (int64_t)p->sl.off[p->sl.k - 1] - (int64_t)p->sl.off[0];
    const int64_t b = 4 * span + 64;
    return b < (int64_t(1) << 31) ? (int32_t)b : 0;
}

bool is_slot_layout(int lanes) { return lanes == FL_ROWS_SLOTS; }
bool is_binned_layout(int lanes) { return lanes == FL_ROWS_BINNED; }

// ---- rows binned by in-degree ----
// A bucket mapping: byte b holds log2 of bucket b's lanes per row (bits 0..2)
// and of its row blocks per tile (bits 3..4).
int map_lanes(uint64_t m, int b) { return 1 << (int)((m >> (8 * b)) & 7u); }
int map_blocks(uint64_t m, int b) { return 1 << (int)((m >> (8 * b + 3)) & 3u); }
int log2i(int v) {
    int l = 0;
    while ((1 << (l + 1)) <= v) ++l;
    return l;
}
uint64_t map_with(uint64_t m, int b, int lanes, int blocks) {
    const uint64_t byte = (uint64_t)(log2i(lanes) | (log2i(blocks) << 3));
    return (m & ~(uint64_t(0xff) << (8 * b))) | (byte << (8 * b));
}
// Largest in-degree of bucket b (the last bucket: taken as 4x its lower edge).
int bucket_hi(int b) { return b == 0 ? 0 : (b == fl::kBuckets - 1 ? 4 << (b - 1) : (1 << b) - 1); }
// Untuned mapping: about a quarter of the bucket's largest in-degree in lanes
// (one round of four loads in flight per lane), one block per tile.
uint64_t default_bin_map() {
    uint64_t m = 0;
    for (int b = 0; b < fl::kBuckets; ++b) {
        int l = 1;
        while (l < 64 && 4 * l < bucket_hi(b)) l <<= 1;
        m = map_with(m, b, l, 1);
    }
    return m;
}
uint64_t bin_map_for(const fl_ctx *ctx, uint64_t shape);

// Classes of a mapping: its distinct (L, T) pairs in ascending order, and the
// class of every bucket.  Returns the number of classes.
int bin_classes(uint64_t m, int8_t *class_of, int *lanes, int *blocks) {
    int n = 0;
    for (int l = 1; l <= 64; l <<= 1)
        for (int t = 1; t <= 8; t <<= 1) {
            bool used = false;
            for (int b = 0; b < fl::kBuckets; ++b)
                if (map_lanes(m, b) == l && map_blocks(m, b) == t) {
                    class_of[b] = (int8_t)n;
                    used = true;
                }
            if (used) {
                lanes[n] = l;
                blocks[n] = t;
                ++n;
            }
        }
    return n;
}

// Bin the rows of `row_ptr` (n rows) into `rows` by the classes of `class_of`;
// sizes[c] receives each class's row count.  Synchronises the stream.
fl_status bin_rows_into(fl_ctx *ctx, const int32_t *row_ptr, int64_t n, const int8_t *class_of, int32_t *rows,
                        int32_t *sizes) {
    const int64_t n_tiles = (n + fl::kBlock - 1) / fl::kBlock;
    int32_t *tmp = pool_alloc<int32_t>(ctx, 2 * fl::kBuckets * n_tiles + fl::kBuckets + 2);
    if (!tmp) return fail(ctx, FL_ENOMEM, "device allocation failed");
    int32_t *d_class = tmp + 2 * fl::kBuckets * n_tiles + fl::kBuckets;
    memcpy(ctx->h_bins, class_of, fl::kBuckets);
    hipStream_t s = ctx->stream;
    hipError_t e = hipMemcpyAsync(d_class, ctx->h_bins, fl::kBuckets, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = fl::launch_bin_rows(row_ptr, (int32_t)n, (const int8_t *)d_class, tmp, tmp + fl::kBuckets * n_tiles,
                                tmp + 2 * fl::kBuckets * n_tiles, rows, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(ctx->h_bins + 16, tmp + 2 * fl::kBuckets * n_tiles, sizeof(int32_t) * fl::kBuckets,
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    ctx->pool.release(tmp);
    if (e != hipSuccess) return fail(ctx, FL_EHIP, "row binning: %s", hipGetErrorString(e));
    memcpy(sizes, ctx->h_bins + 16, sizeof(int32_t) * fl::kBuckets);
    return FL_OK;
}

// Table of classes over binned rows: rows[c] rows in class c (in order),
// lanes and blocks per class; empty classes are left out.
fl::BinTable bin_table(int n_classes, const int32_t *rows, const int *lanes, const int *blocks) {
    fl::BinTable t{};
    int32_t row = 0, tile = 0;
    for (int c = 0; c < n_classes; ++c) {
        if (rows[c] > 0) {
            fl::BinClass &k = t.c[t.n_classes++];
            k.row_begin = row;
            k.rows = rows[c];
            k.tile_begin = tile;
            k.lanes = (int16_t)lanes[c];
            k.blocks = (int16_t)blocks[c];
            const int32_t per = blocks[c] * (fl::kBlock / lanes[c]);
            tile += (rows[c] + per - 1) / per;
        }
        row += rows[c];
    }
    t.tiles = tile;
    return t;
}

// The plan's rows binned for mapping m (kept while batch members sweep them).
fl_status ensure_binned(fl_ctx *ctx, fl_plan *p, uint64_t m) {
    if (p->have_bins && (p->bin_map == m || p->bin_users > 0)) return FL_OK;
    int8_t class_of[fl::kBuckets];
    int lanes[fl::kBuckets], blocks[fl::kBuckets];
    const int nc = bin_classes(m, class_of, lanes, blocks);
    if (!p->bin_rows) {
        p->bin_rows = pool_alloc<int32_t>(ctx, p->n);
        if (!p->bin_rows) return fail(ctx, FL_ENOMEM, "device allocation failed");
    }
    int32_t sizes[fl::kBuckets];
    const fl_status st = bin_rows_into(ctx, p->row_ptr, p->n, class_of, p->bin_rows, sizes);
    if (st != FL_OK) return st;
    p->bins = bin_table(nc, sizes, lanes, blocks);
    p->bin_map = m;
    p->have_bins = true;
    return FL_OK;
}

struct Resolved {
    double d, p, tol;
    int32_t max_iter;
    int lanes;  // FL_ROWS_SLOTS or CSR lanes
    bool lag;   // lagged step (no FL_STEP_SEPARATE)
};

fl_status resolve_params(fl_ctx *ctx, const fl_plan *p, const fl_params *prm, Resolved &r, bool exact = false) {
    const double d = prm->damping;
    if (exact ? !(d > 0.0 && d <= 1.0) : !(d > 0.0 && d < 1.0))
        return fail(ctx, FL_EINVAL, exact ? "damping must be in (0,1]" : "damping must be in (0,1)");
    if (!(prm->p >= 0.0) || !isfinite(prm->p)) return fail(ctx, FL_EINVAL, "p must be finite and >= 0");
    if (!(prm->tol_l1 >= 0.0) || !isfinite(prm->tol_l1)) return fail(ctx, FL_EINVAL, "tol_l1 must be finite and >= 0");
    if (prm->max_iter < 0) return fail(ctx, FL_EINVAL, "max_iter must be >= 0");
    if (prm->flags & ~FL_STEP_SEPARATE) return fail(ctx, FL_EINVAL, "unknown flags 0x%x", prm->flags);
    if (prm->reserved != 0) return fail(ctx, FL_EINVAL, "reserved must be 0");
    if (prm->row_mapping != 0 && !is_slot_layout(prm->row_mapping) && !is_binned_layout(prm->row_mapping) &&
        !valid_lanes(prm->row_mapping))
        return fail(ctx, FL_EINVAL, "row_mapping must be 0, FL_ROWS_SLOTS, FL_ROWS_BINNED or a power of two <= 64");
    if (is_slot_layout(prm->row_mapping) && p->sl.words == 0)
        return fail(ctx, FL_EINVAL, "the slot sweep needs at most %d candidate slots (space has %d)",
                    fl::kMaxSlots, p->sl.k);
    r.d = d;
    r.p = prm->p;
    r.tol = prm->tol_l1 > 0.0 ? prm->tol_l1 : 2e-7;
    // the exact sweeps settle after (longest path + 1) <= N sweeps
    r.max_iter = prm->max_iter > 0 ? prm->max_iter : (exact ? (int32_t)std::min<int64_t>(p->n + 2, INT32_MAX) : 1000);
    r.lanes = prm->row_mapping ? prm->row_mapping : (p->sl.words > 0 ? FL_ROWS_SLOTS : FL_ROWS_BINNED);
    r.lag = !(prm->flags & FL_STEP_SEPARATE);
    return FL_OK;
}

// y, x (x in raw-index space for the slot sweep) and the state of a plan;
// lag: the third y buffer and g of the lagged step as well.
fl_status ensure_pr_buffers(fl_ctx *ctx, fl_plan *p, bool slots, bool lag) {
    if (!p->state) {
        for (int j = 0; j < 2; ++j) p->y[j] = pool_alloc<float>(ctx, p->n);
        p->state = pool_alloc<PrState>(ctx, 1);
        if (!p->y[0] || !p->y[1] || !p->state) return fail(ctx, FL_ENOMEM, "device allocation failed");
    }
    if (lag && !p->g) {
        p->y[2] = pool_alloc<float>(ctx, p->n);
        p->g = pool_alloc<float>(ctx, p->n);
        if (!p->y[2] || !p->g) return fail(ctx, FL_ENOMEM, "device allocation failed");
    }
    const int64_t x_need = slots ? (p->n_raw + 3) / 4 * 4 : p->n;   // raw-index space, whole 16-byte groups
    if (x_need > p->x_cap) {
        for (int j = 0; j < 2; ++j) {
            ctx->pool.release(p->x[j]);
            p->x[j] = pool_alloc<float>(ctx, x_need);
        }
        if (!p->x[0] || !p->x[1]) return fail(ctx, FL_ENOMEM, "device allocation failed");
        p->x_cap = x_need;
    }
    return FL_OK;
}

int32_t tiles_of(const fl_plan *p) { return (int32_t)((p->n + fl::kBlock - 1) / fl::kBlock); }

fl_status ensure_partials(fl_ctx *ctx, fl_plan *p, int64_t triples) {
    if (triples <= p->pr_grid) return FL_OK;
    ctx->pool.release(p->partials);
    p->partials = pool_alloc<double>(ctx, 3 * triples);
    if (!p->partials) {
        p->pr_grid = 0;
        return fail(ctx, FL_ENOMEM, "device allocation failed");
    }
    p->pr_grid = (int)triples;
    return FL_OK;
}



void fill_summary(const fl_plan *p, const PrState &hs, int lanes, fl_status status, fl_summary *out) {
    fill_sizes(p, out);
    out->iterations = hs.k;
    out->row_mapping = lanes;
    out->status = status;
    out->residual_l1 = hs.resid;
    out->mass_minima = hs.score_den;
    out->mass_near = hs.score_num;
    out->score = hs.score_den > 0.0 ? hs.score_num / hs.score_den : 0.0;
}

// Shape class of a plan for the tuning cache: record width, neighbourhood,
// log2 N and the mean in-degree rounded to a half.
uint64_t shape_key(const fl_plan *p) {
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= p->n) ++lg;
    const int64_t deg2 = p->n > 0 ? (2 * p->e + p->n / 2) / p->n : 0;
    return ((uint64_t)p->sl.words << 56) | ((uint64_t)p->adjacent << 52) | ((uint64_t)lg << 40) |
           (uint64_t)std::min<int64_t>(deg2, (int64_t(1) << 40) - 1);
}

uint64_t bin_map_for(const fl_ctx *ctx, uint64_t shape) {
    const auto it = ctx->tuned_map.find(shape);
    return it != ctx->tuned_map.end() ? it->second : default_bin_map();
}

// Grid, buffers and arguments of the power iteration of plan p in layout
// `lanes` (FL_ROWS_SLOTS or CSR lanes per row).
fl_status prepare_pr(fl_ctx *ctx, fl_plan *p, const Resolved &r, int lanes, PrArgs &a, int &grid,
                     int &init_grid) {
    const int kind = is_slot_layout(lanes) ? fl::kSweepSlots : is_binned_layout(lanes) ? fl::kSweepBinned
                                                                                      : fl::kSweepCsr;
    a = PrArgs{};
    a.kind = kind;
    if (kind == fl::kSweepBinned) {
        const fl_status bst = ensure_binned(ctx, p, bin_map_for(ctx, shape_key(p)));
        if (bst != FL_OK) return bst;
        a.bin_rows = p->bin_rows;
        a.bins = p->bins;
    }
    a.adjacent = p->adjacent;
    a.x_bytes = kind == fl::kSweepSlots ? x_bytes_of(p) : 0;
    // persistent grid: every workgroup resident at once (occupancy query), a
    // multiple of the XCD count so each XCD gets the same number of them
    int per_cu = 0;
    FL_HIP(fl::pr_iter_blocks_per_cu(a, p->sp, p->sl, lanes, &per_cu));
    const int64_t resident =
        std::max<int64_t>(fl::kXcds, (int64_t)std::max(per_cu, 1) * ctx->num_cus / fl::kXcds * fl::kXcds);
    const int64_t rows_per_wg = kind == fl::kSweepSlots ? fl::kBlock : (kind == fl::kSweepBinned ? 1 : fl::kBlock / lanes);
    const int64_t groups = kind == fl::kSweepBinned ? std::max<int64_t>(p->bins.tiles, 1)
                                                    : (p->n + rows_per_wg - 1) / rows_per_wg;
    grid = (int)std::min<int64_t>(resident, (groups + fl::kXcds - 1) / fl::kXcds * fl::kXcds);
    fl_status st = ensure_pr_buffers(ctx, p, kind == fl::kSweepSlots, r.lag);
    if (st != FL_OK) return st;
    // partial sums: one triple per tile (init, slot sweep) or per workgroup
    // (CSR sweep, lagged step: two buffers of them)
    const int32_t n_tiles = tiles_of(p);
    init_grid = (int)std::min<int64_t>(n_tiles, (int64_t)ctx->num_cus * 4);
    st = ensure_partials(ctx, p, std::max<int64_t>(std::max<int64_t>(2 * (int64_t)grid, n_tiles), p->have_bins ? p->bins.tiles : 0));
    if (st != FL_OK) return st;
    a.row_ptr = p->row_ptr;
    a.col_idx = p->col_idx;
    a.out_deg = p->out_deg;
    a.valid_raw = p->valid_raw;
    a.rec = p->rec;
    a.presence = p->presence;
    a.k_pad = k_pad_of(p->sl);
    a.off = p->d_off;
    a.k_slots = p->sl.k;
    a.y[0] = p->y[0];
    a.y[1] = p->y[1];
    a.y[2] = p->y[2];
    a.g = p->g;
    a.lag = r.lag ? 1 : 0;
    a.sweep = 0;
    a.n_parts = grid;
    a.part_stride = grid;
    a.n_sinks = p->m;
    a.x[0] = p->x[0];
    a.x[1] = p->x[1];
    a.partials = p->partials;
    a.st = p->state;
    a.n = (int32_t)p->n;
    a.d = r.d;
    a.tol = r.tol;
    a.max_iter = r.max_iter;
    return FL_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Batches: members swept together by the segmented kernels, joining and
// leaving at step boundaries (continuous batching).

struct fl_batch {
    struct Member {
        fl_plan *plan = nullptr;
        Resolved prm{};
        double *out_pr = nullptr;
        int32_t *out_min = nullptr;
        int64_t tag = 0;
        int slot = -1;    // row of the device member table
        int phase = 0;    // 0 waiting for initialisation, 1 running, 2 finished
        fl_summary sum{};
        bool binned = false;  // binned sweep over the CSR (else the slot sweep)
        bool holds_bins = false;  // counted in plan->bin_users
        // the member's own iterate: y (node ids), x (raw indices; node ids
        // when binned), per-tile partial sums and state, from the context's pool
        float *y[2] = {}, *x[2] = {};
        double *partials = nullptr;
        PrState *state = nullptr;
    };
    fl_ctx *ctx = nullptr;
    std::vector<Member> members;
    std::vector<int> free_slots;
    int capacity = 0;
    fl::BatchMember *d_members = nullptr, *h_members = nullptr;
    fl::TileRef *d_tiles = nullptr, *h_tiles = nullptr;  // regions: init | sweep | output
    int64_t tile_cap = 0;
    int32_t *d_ids = nullptr, *h_ids = nullptr;  // regions: init | running | finishing
    PrState *d_states = nullptr, *h_states = nullptr;
    // list ranges read by the sweep and step kernels: [2w], [2w+1] start and
    // length of the tiles of record width w (1..kMaxWords; 0: binned
    // members) in the sweep list, [kRunCount] running members, [kInitCount]
    // joining ones
    static constexpr int kRunCount = 2 * fl::kMaxWords + 2, kInitCount = kRunCount + 1, kCounts = 16;
    int32_t *d_counts = nullptr, *h_counts = nullptr;
    int sweep_per_cu[fl::kMaxWords + 1] = {};
    int64_t sweeps = 0;
    double sweep_ms = 0.0;
    hipEvent_t ev[2] = {};
    // the captured sweep loop of one step, per launch shape (kept for the
    // shapes seen recently, so membership moving back and forth between
    // shapes replays instead of recapturing; dropped when the tables move)
    bool use_graphs = true;
    hipStream_t capture_stream = nullptr;  // private, only ever captured (the context's stream may be the null stream)
    // members of at most small_tiles tiles (0: none) iterate in one workgroup
    // each, on a second stream of the same priority, alongside the others
    int32_t small_tiles = fl::kSmallTiles;
    hipStream_t side_stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    struct Shape {
        int32_t sweeps = 0, finish_grid = 0;
        int32_t grid[fl::kMaxWords + 1] = {};
        const void *members = nullptr, *tiles = nullptr, *ids = nullptr;
        bool operator==(const Shape &o) const {
            if (sweeps != o.sweeps || finish_grid != o.finish_grid || members != o.members || tiles != o.tiles ||
                ids != o.ids)
                return false;
            for (int w = 0; w <= fl::kMaxWords; ++w)
                if (grid[w] != o.grid[w]) return false;
            return true;
        }
    };
    static constexpr size_t kMaxGraphs = 256;
    std::vector<std::pair<Shape, hipGraphExec_t>> graphs;   // least recently used first
    int64_t graph_launches = 0, graph_captures = 0;
};

namespace {

// Tiles a member needs in the batch's lists: node tiles (initial iterate,
// output) and, when binned, the tiles of its bin table (sweeps).
int64_t member_tiles(const fl_batch::Member &m) {
    return std::max<int64_t>(tiles_of(m.plan), m.binned ? m.plan->bins.tiles : 0);
}

void member_release(fl_ctx *ctx, fl_batch::Member &m) {
    if (m.holds_bins) {
        m.plan->bin_users -= 1;
        m.holds_bins = false;
    }
    for (int j = 0; j < 2; ++j) {
        ctx->pool.release(m.y[j]);
        ctx->pool.release(m.x[j]);
        m.y[j] = m.x[j] = nullptr;
    }
    ctx->pool.release(m.partials);
    ctx->pool.release(m.state);
    m.partials = nullptr;
    m.state = nullptr;
}

fl_status member_alloc(fl_ctx *ctx, const fl_plan *p, fl_batch::Member &m) {
    // one block, based at y[0]
    const int64_t nx = m.binned ? p->n : (p->n_raw + 3) / 4 * 4;
    Carve c;
    c.add(m.y[0], p->n).add(m.y[1], p->n).add(m.x[0], nx).add(m.x[1], nx);
    c.add(m.partials, 3 * std::max<int64_t>(tiles_of(p), m.binned ? p->bins.tiles : 0)).add(m.state, 1).take(ctx);
    if (!m.y[0] || !m.y[1] || !m.x[0] || !m.x[1] || !m.partials || !m.state) {
        member_release(ctx, m);
        return fail(ctx, FL_ENOMEM, "device allocation failed");
    }
    return FL_OK;
}

// Destroy the batch's captured graphs (their kernel arguments point at the
// batch tables, so they go whenever the tables are reallocated).
void batch_free_graphs(fl_batch *b) {
    for (auto &g : b->graphs) (void)hipGraphExecDestroy(g.second);
    b->graphs.clear();
}

void batch_free_tables(fl_batch *b) {
    batch_free_graphs(b);
    fl_ctx *ctx = b->ctx;
    ctx->pool.release(b->d_members);
    ctx->pool.release(b->d_tiles);
    ctx->pool.release(b->d_ids);
    ctx->pool.release(b->d_states);
    if (b->h_members) (void)hipHostFree(b->h_members);
    if (b->h_tiles) (void)hipHostFree(b->h_tiles);
    if (b->h_ids) (void)hipHostFree(b->h_ids);
    if (b->h_states) (void)hipHostFree(b->h_states);
    b->d_members = b->h_members = nullptr;
    b->d_tiles = b->h_tiles = nullptr;
    b->d_ids = b->h_ids = nullptr;
    b->d_states = b->h_states = nullptr;
}

// Member table, id lists and state snapshots for `cap` members and `tiles`
// tiles (three regions each).  Only called between steps.
// Pinned segment tables of the segmented build: room for `segs` spaces and
// `tiles` tile entries (grown, never shrunk; freed with the context).
fl_status seg_tables_reserve(fl_ctx *ctx, int32_t segs, int64_t tiles) {
    if (segs > ctx->seg_cap) {
        (void)hipHostFree(ctx->h_segs);
        (void)hipHostFree(ctx->h_seg_ids);
        (void)hipHostFree(ctx->h_seg_sizes);
        ctx->h_segs = nullptr;
        ctx->h_seg_ids = nullptr;
        ctx->h_seg_sizes = nullptr;
        ctx->seg_cap = 0;
        const int32_t cap = std::max(segs, 64);
        if (hipHostMalloc((void **)&ctx->h_segs, sizeof(fl::SegBuild) * cap, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&ctx->h_seg_ids, sizeof(int32_t) * cap, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&ctx->h_seg_sizes, sizeof(BuildSizes) * cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return FL_ENOMEM;
        }
        ctx->seg_cap = cap;
    }
    if (tiles > ctx->seg_tile_cap) {
        const int64_t cap = std::max<int64_t>(tiles, 2 * ctx->seg_tile_cap + 4096);
        (void)hipHostFree(ctx->h_seg_tiles);
        ctx->h_seg_tiles = nullptr;
        ctx->seg_tile_cap = 0;
        if (hipHostMalloc((void **)&ctx->h_seg_tiles, sizeof(fl::SegTile) * cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return FL_ENOMEM;
        }
        ctx->seg_tile_cap = cap;
    }
    return FL_OK;
}

fl_status batch_reserve(fl_batch *b, int cap, int64_t tiles) {
    fl_ctx *ctx = b->ctx;
    if (cap <= b->capacity && tiles <= b->tile_cap) return FL_OK;
    const int new_cap = std::max(cap, std::max(16, 2 * b->capacity));
    const int64_t new_tiles = std::max<int64_t>(tiles, std::max<int64_t>(1024, 2 * b->tile_cap));
    fl::BatchMember *dm = pool_alloc<fl::BatchMember>(ctx, new_cap);
    fl::TileRef *dt = pool_alloc<fl::TileRef>(ctx, 3 * new_tiles);
    int32_t *di = pool_alloc<int32_t>(ctx, 3 * (int64_t)new_cap);
    PrState *ds = pool_alloc<PrState>(ctx, new_cap);
    fl::BatchMember *hm = nullptr;
    fl::TileRef *ht = nullptr;
    int32_t *hi = nullptr;
    PrState *hs = nullptr;
    if (!dm || !dt || !di || !ds ||
        hipHostMalloc((void **)&hm, sizeof(fl::BatchMember) * new_cap, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&ht, sizeof(fl::TileRef) * 3 * new_tiles, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&hi, sizeof(int32_t) * 3 * new_cap, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&hs, sizeof(PrState) * new_cap, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        ctx->pool.release(dm);
        ctx->pool.release(dt);
        ctx->pool.release(di);
        ctx->pool.release(ds);
        if (hm) (void)hipHostFree(hm);
        if (ht) (void)hipHostFree(ht);
        if (hi) (void)hipHostFree(hi);
        if (hs) (void)hipHostFree(hs);
        return fail(ctx, FL_ENOMEM, "batch tables: allocation failed");
    }
    if (b->h_members) memcpy(hm, b->h_members, sizeof(fl::BatchMember) * b->capacity);
    batch_free_tables(b);
    b->d_members = dm;
    b->h_members = hm;
    b->d_tiles = dt;
    b->h_tiles = ht;
    b->d_ids = di;
    b->h_ids = hi;
    b->d_states = ds;
    b->h_states = hs;
    for (int j = b->capacity; j < new_cap; ++j) b->free_slots.push_back(j);
    b->capacity = new_cap;
    b->tile_cap = new_tiles;
    return FL_OK;
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
        hipHostMalloc((void **)&ctx->h_state, sizeof(PrState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_bins, sizeof(int32_t) * 64, hipHostMallocDefault) != hipSuccess ||
        scratch_address(device, &ctx->scratch) != hipSuccess) {
        (void)hipGetLastError();
        if (ctx->h_sizes) (void)hipHostFree(ctx->h_sizes);
        if (ctx->h_state) (void)hipHostFree(ctx->h_state);
        if (ctx->h_bins) (void)hipHostFree(ctx->h_bins);
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
    if (ctx->analyze_batch) (void)fl_batch_destroy(ctx, ctx->analyze_batch);
    (void)hipHostFree(ctx->h_segs);
    (void)hipHostFree(ctx->h_seg_tiles);
    (void)hipHostFree(ctx->h_seg_ids);
    (void)hipHostFree(ctx->h_seg_sizes);
    ctx->pool.release_all();
    for (hipEvent_t e : ctx->sweep_ev) (void)hipEventDestroy(e);
    (void)hipHostFree(ctx->h_sizes);
    (void)hipHostFree(ctx->h_state);
    (void)hipHostFree(ctx->h_bins);
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
    if (!out) return fail(ctx, FL_EINVAL, "null argument");
    *out = nullptr;
    FL_HIP(hipSetDevice(ctx->device));
    Build b;
    b.h_sizes = ctx->h_sizes;
    auto sync = [&]() {
        if (b.status != FL_OK) return;
        hipError_t he = hipStreamSynchronize(ctx->stream);
        if (he != hipSuccess) build_fail(b, FL_EHIP, "%s", hipGetErrorString(he));
    };
    build_begin(ctx, b, space, d_fitness_raw, nb);
    sync();
    build_degree(ctx, b);
    sync();
    build_fill(ctx, b);
    (void)hipStreamSynchronize(ctx->stream);
    build_end(ctx, b);
    if (b.status != FL_OK) {
        build_abort(ctx, b);
        return fail(ctx, b.status, "%s", b.err.c_str());
    }
    if (b.p->sl.words == 0) {
        // no slot records: the binned sweep is this plan's layout, so its rows
        // are binned now (a plan may join a batch of another context, which
        // must not allocate from this one)
        const fl_status bst = ensure_binned(ctx, b.p, bin_map_for(ctx, shape_key(b.p)));
        if (bst != FL_OK) {
            const std::string msg = ctx->err;
            build_abort(ctx, b);
            return fail(ctx, bst, "%s", msg.c_str());
        }
    }
    if (sizes) fill_sizes(b.p, sizes);
    *out = b.p;
    return FL_OK;
}

namespace {

// PageRank, minima and C_p of a built plan.  quiet: no timing events are
// created or recorded and no sweep is profiled (fl_analyze_noalloc).
fl_status execute_impl(fl_ctx *ctx, fl_plan *p, const fl_params *prm, double *d_pagerank, int32_t *d_minima,
                       fl_summary *out, bool exact, bool quiet = false) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!p || !prm || !d_pagerank || (!d_minima && p->m > 0)) return fail(ctx, FL_EINVAL, "null argument");
    if (p->ctx != ctx) return fail(ctx, FL_EINVAL, "plan belongs to another context");
    Resolved r;
    fl_status st = resolve_params(ctx, p, prm, r, exact);
    if (st != FL_OK) return st;
    int lanes = r.lanes;
    if (prm->row_mapping == 0) {
        const auto hit = ctx->tuned.find(shape_key(p));
        if (hit != ctx->tuned.end()) lanes = hit->second;
    }
    FL_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    PrArgs a;
    int grid = 0, init_grid = 0;
    st = prepare_pr(ctx, p, r, lanes, a, grid, init_grid);
    if (st != FL_OK) return st;
    a.exact = exact ? 1 : 0;
    const bool timed = !quiet;
    const int32_t profile_every = quiet ? 0 : ctx->profile_every;
    if (timed) FL_HIP(ensure_events(p));

    if (timed) FL_HIP(hipEventRecord(p->ev[2], s));
    FL_HIP(hipMemsetAsync(p->state, 0, sizeof(PrState), s));
    FL_HIP(fl::launch_pr_init(a, init_grid, s));

    // Launch the iteration kernel in chunks; a launch after convergence exits
    // at once.  The chunk length follows the observed residual decay so that
    // few host round trips and few empty launches are needed.  With the
    // lagged step the sweeps alone are launched, and the step of iteration k
    // runs in sweep k + 1 (k + 2 for the power iteration, whose residual is
    // one sweep late as well): the sweep after the cap's last iteration does
    // only that step, and sets the stop flag.
    int launches = 0;
    int chunk = 16;
    const int64_t limit = r.lag ? (int64_t)r.max_iter + (exact ? 1 : 2) : INT64_MAX;
    double iterate_ms = 0.0, sweep_ms = 0.0;
    PrState *hs = ctx->h_state;
    int sampled = 0;
    for (;;) {
        if (profile_every > 0 && (int)ctx->sweep_ev.size() < 2 * chunk) {
            for (int j = (int)ctx->sweep_ev.size(); j < 2 * chunk; ++j) {
                hipEvent_t e;
                FL_HIP(hipEventCreate(&e));
                ctx->sweep_ev.push_back(e);
            }
        }
        if (timed) FL_HIP(hipEventRecord(p->ev[5], s));
        for (int j = 0; j < chunk; ++j) {
            const bool sampled_here = profile_every > 0 && (launches + j) % profile_every == 0;
            a.sweep = launches + j;
            if (sampled_here) FL_HIP(hipEventRecord(ctx->sweep_ev[2 * j], s));
            FL_HIP(fl::launch_pr_sweep(a, p->sl, lanes, grid, s));
            if (sampled_here) FL_HIP(hipEventRecord(ctx->sweep_ev[2 * j + 1], s));
            FL_HIP(fl::launch_pr_step(a, grid, s));
        }
        if (timed) FL_HIP(hipEventRecord(p->ev[6], s));
        const int before = launches;
        launches += chunk;
        FL_HIP(hipMemcpyAsync(hs, p->state, sizeof(PrState), hipMemcpyDeviceToHost, s));
        FL_HIP(hipStreamSynchronize(s));
        if (timed) iterate_ms += elapsed(p->ev[5], p->ev[6]);
        if (profile_every > 0)   // launches past the converged iteration exit at once: not counted
            for (int j = 0; j < chunk && before + j < hs->worked; ++j)
                if ((before + j) % profile_every == 0) {
                    sweep_ms += elapsed(ctx->sweep_ev[2 * j], ctx->sweep_ev[2 * j + 1]);
                    ++sampled;
                }
        if (hs->done) break;
        if (launches >= limit) return fail(ctx, FL_EHIP, "the iteration did not stop after %d sweeps", launches);
        const double rate = (hs->resid_prev > 0.0) ? hs->resid / hs->resid_prev : 1.0;
        if (exact) {
            chunk = 64;   // the sweeps end abruptly (exact fixed point): no decay to follow
        } else if (rate > 0.0 && rate < 0.999 && hs->resid > r.tol) {
            const double more = ceil(log(r.tol / hs->resid) / log(rate));
            chunk = (int)std::min(64.0, std::max(2.0, more + 1.0));
        } else {
            chunk = 8;
        }
        chunk = std::min(chunk, std::max(1, r.max_iter - hs->k));
        if (r.lag) chunk = (int)std::min<int64_t>(chunk, limit - launches);
    }
    if (timed) FL_HIP(hipEventRecord(p->ev[3], s));
    FL_HIP(fl::launch_pr_output(a, d_pagerank, s));
    if (p->m > 0) FL_HIP(hipMemcpyAsync(d_minima, p->minima, sizeof(int32_t) * p->m, hipMemcpyDeviceToDevice, s));
    const double threshold = (1.0 + r.p) * (double)p->f_opt;
    FL_HIP(fl::launch_score(d_pagerank, p->minima, (int32_t)p->m, p->fit_c, threshold, p->state, s));
    if (timed) FL_HIP(hipEventRecord(p->ev[4], s));
    FL_HIP(hipMemcpyAsync(hs, p->state, sizeof(PrState), hipMemcpyDeviceToHost, s));
    FL_HIP(hipStreamSynchronize(s));

    p->timing.pagerank_ms = timed ? elapsed(p->ev[2], p->ev[3]) : 0.0;
    p->timing.score_ms = timed ? elapsed(p->ev[3], p->ev[4]) : 0.0;
    p->timing.iterate_ms = iterate_ms;
    p->timing.sweep_ms = sweep_ms;
    p->timing.sweeps_timed = sampled;
    p->timing.iterations = hs->worked;
    p->timing.launches = launches;
    const fl_status result = hs->done == 1 ? FL_OK : FL_ENOCONV;
    if (out) fill_summary(p, *hs, lanes, result, out);
    if (result != FL_OK)
        return fail(ctx, FL_ENOCONV, "no convergence after %d iterations (residual %.3e)", hs->k, hs->resid);
    return FL_OK;
}

}  // namespace

fl_status fl_execute(fl_ctx *ctx, fl_plan *p, const fl_params *prm, double *d_pagerank, int32_t *d_minima,
                     fl_summary *out) {
    return execute_impl(ctx, p, prm, d_pagerank, d_minima, out, false);
}

fl_status fl_execute_exact(fl_ctx *ctx, fl_plan *p, const fl_params *prm, double *d_pagerank, int32_t *d_minima,
                           fl_summary *out) {
    return execute_impl(ctx, p, prm, d_pagerank, d_minima, out, true);
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

fl_status fl_score_curve(fl_ctx *ctx, const fl_plan *p, const double *d_pagerank, int32_t n_p,
                         const double *p_values, double *scores) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!p || p->ctx != ctx || !d_pagerank || !p_values || !scores) return fail(ctx, FL_EINVAL, "bad argument");
    if (n_p < 1 || n_p > 4096) return fail(ctx, FL_EINVAL, "n_p must be in [1, 4096]");
    for (int32_t j = 0; j < n_p; ++j)
        if (!(p_values[j] >= 0.0) || !isfinite(p_values[j])) return fail(ctx, FL_EINVAL, "p must be finite and >= 0");
    FL_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    double *h = nullptr;   // thresholds, then num/den pairs
    if (hipHostMalloc((void **)&h, sizeof(double) * 3 * (size_t)n_p, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, FL_ENOMEM, "pinned allocation failed");
    }
    double *d = pool_alloc<double>(ctx, 3 * (int64_t)n_p);
    if (!d) {
        (void)hipHostFree(h);
        return fail(ctx, FL_ENOMEM, "device allocation failed");
    }
    for (int32_t j = 0; j < n_p; ++j) h[j] = (1.0 + p_values[j]) * (double)p->f_opt;
    hipError_t e = hipMemcpyAsync(d, h, sizeof(double) * n_p, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = fl::launch_score_curve(d_pagerank, p->minima, (int32_t)p->m, p->fit_c, d, n_p, d + n_p, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h + n_p, d + n_p, sizeof(double) * 2 * n_p, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        for (int32_t j = 0; j < n_p; ++j) scores[j] = h[n_p + 2 * j] / h[n_p + 2 * j + 1];
    ctx->pool.release(d);
    (void)hipHostFree(h);
    if (e != hipSuccess) return fail(ctx, FL_EHIP, "C_p curve: %s", hipGetErrorString(e));
    return FL_OK;
}

fl_status fl_naive_metric(fl_ctx *ctx, const fl_plan *p, double *d_ratio, int32_t n_bins, int64_t *hist) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!p || p->ctx != ctx) return fail(ctx, FL_EINVAL, "bad plan");
    if (n_bins < 1 || n_bins > 65536) return fail(ctx, FL_EINVAL, "n_bins must be in [1, 65536]");
    FL_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    double *ratio = d_ratio ? d_ratio : pool_alloc<double>(ctx, std::max<int64_t>(p->m, 1));
    uint32_t *dh = pool_alloc<uint32_t>(ctx, n_bins);
    uint32_t *hh = nullptr;
    if (!ratio || !dh ||
        hipHostMalloc((void **)&hh, sizeof(uint32_t) * (size_t)n_bins, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        if (!d_ratio) ctx->pool.release(ratio);
        ctx->pool.release(dh);
        return fail(ctx, FL_ENOMEM, "allocation failed");
    }
    hipError_t e = fl::launch_naive(p->minima, (int32_t)p->m, p->fit_c, p->f_opt, ratio, n_bins, dh, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hh, dh, sizeof(uint32_t) * n_bins, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && hist)
        for (int32_t j = 0; j < n_bins; ++j) hist[j] = hh[j];
    if (!d_ratio) ctx->pool.release(ratio);
    ctx->pool.release(dh);
    (void)hipHostFree(hh);
    if (e != hipSuccess) return fail(ctx, FL_EHIP, "naive metric: %s", hipGetErrorString(e));
    return FL_OK;
}

fl_status fl_profile(fl_ctx *ctx, int32_t every) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (every < 0) return fail(ctx, FL_EINVAL, "every must be >= 0");
    ctx->profile_every = every;
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
    plan_free(p);
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
        const std::string msg = ctx->err;
        const fl_status xs = fl_plan_export(ctx, p, d_valid_raw, nullptr, nullptr, nullptr);
        if (xs != FL_OK) st = xs;
        else ctx->err = msg;
    }
    const std::string msg = ctx->err;
    fl_plan_destroy(ctx, p);
    ctx->err = msg;
    return st;
}

fl_status fl_analyze_noalloc(fl_ctx *ctx, const fl_space *space, const float *d_fitness_raw, fl_neighbourhood nb,
                             const fl_params *params, double *d_pagerank, int32_t *d_minima, int32_t *d_valid_raw,
                             fl_summary *out) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!space || !space->radix || !d_fitness_raw || !params || !d_pagerank || !d_minima)
        return fail(ctx, FL_EINVAL, "null argument");
    if (!ctx->scratch) return fail(ctx, FL_EHIP, "no scratch array on device %d", ctx->device);
    // Before any launch: the buffers sized by the raw space alone (node map,
    // compacted fitness, remap, two x vectors) must fit.
    int64_t n_raw = 1;
    for (int i = 0; i < space->n_params && i < fl::kMaxParams; ++i) {
        n_raw *= std::max<int32_t>(space->radix[i], 1);
        if (n_raw >= (int64_t(1) << 31)) break;
    }
    const int64_t raw_bytes = 20 * n_raw;
    if (raw_bytes > (int64_t)kNoAllocScratchBytes)
        return fail(ctx, FL_EINVAL,
                    "fl_analyze_noalloc: a space of %lld configurations needs at least %lld bytes of scratch, "
                    "more than its %zu bytes; use fl_analyze",
                    (long long)n_raw, (long long)raw_bytes, kNoAllocScratchBytes);
    FL_HIP(hipSetDevice(ctx->device));
    Arena arena;
    arena.base = static_cast<char *>(ctx->scratch);
    arena.cap = kNoAllocScratchBytes;
    ctx->arena = &arena;
    fl_plan plan;   // built in place: no host allocation either
    Build b;
    b.h_sizes = ctx->h_sizes;
    b.timed = false;
    b.storage = &plan;
    auto sync = [&]() {
        if (b.status != FL_OK) return;
        hipError_t he = hipStreamSynchronize(ctx->stream);
        if (he != hipSuccess) build_fail(b, FL_EHIP, "%s", hipGetErrorString(he));
    };
    build_begin(ctx, b, space, d_fitness_raw, nb);
    sync();
    build_degree(ctx, b);
    sync();
    build_fill(ctx, b);
    (void)hipStreamSynchronize(ctx->stream);
    build_end(ctx, b);
    fl_status st = b.status;
    if (st == FL_OK) {
        st = execute_impl(ctx, &plan, params, d_pagerank, d_minima, out, false, true);
        if ((st == FL_OK || st == FL_ENOCONV) && d_valid_raw) {
            const hipError_t he = hipMemcpyAsync(d_valid_raw, plan.valid_raw, 4 * plan.n, hipMemcpyDeviceToDevice,
                                                 ctx->stream);
            const hipError_t hs = hipStreamSynchronize(ctx->stream);
            if (he != hipSuccess || hs != hipSuccess) st = fail(ctx, FL_EHIP, "node map copy failed");
        }
    } else {
        (void)hipStreamSynchronize(ctx->stream);
        fail(ctx, st, "%s", b.err.c_str());
    }
    ctx->arena = nullptr;
    if (arena.overflow)
        st = fail(ctx, FL_EINVAL,
                  "fl_analyze_noalloc: the space's FFG and iterates need more than the %zu bytes of scratch; "
                  "use fl_analyze",
                  kNoAllocScratchBytes);
    return st;
}

}  // extern "C"

namespace {

// Rows of plan p grouped by in-degree bucket (every bucket its own class)
// into rows (N entries); sizes[b] receives each bucket's row count.
fl_status bucket_rows(fl_ctx *ctx, const fl_plan *p, int32_t *rows, int32_t *sizes) {
    int8_t ident[fl::kBuckets];
    for (int b = 0; b < fl::kBuckets; ++b) ident[b] = (int8_t)b;
    return bin_rows_into(ctx, p->row_ptr, p->n, ident, rows, sizes);
}

// The per-bucket part of the autotuner: for every non-empty in-degree bucket,
// time `sweeps` binned sweeps over that bucket's rows alone for every lanes
// per row L up to the bucket's largest in-degree (rounded up to a power of
// two) and T in {1, 4} blocks per tile; *map receives the fastest (L, T) of
// each bucket (the default for empty buckets).
fl_status tune_buckets(fl_ctx *ctx, fl_plan *p, const Resolved &r, int32_t sweeps, uint64_t *map) {
    hipStream_t s = ctx->stream;
    int32_t *rows = pool_alloc<int32_t>(ctx, p->n);
    if (!rows) return fail(ctx, FL_ENOMEM, "device allocation failed");
    int32_t sizes[fl::kBuckets];
    fl_status st = bucket_rows(ctx, p, rows, sizes);
    PrArgs a;
    int grid = 0, init_grid = 0;
    if (st == FL_OK) st = prepare_pr(ctx, p, r, FL_ROWS_BINNED, a, grid, init_grid);
    // partial triples of the largest candidate table (64 lanes, one block)
    if (st == FL_OK) st = ensure_partials(ctx, p, p->n / 4 + fl::kBuckets + 1);
    int per_cu = 0;
    if (st == FL_OK && fl::pr_binned_blocks_per_cu(&per_cu) != hipSuccess) st = fail(ctx, FL_EHIP, "occupancy query");
    uint64_t m = default_bin_map();
    if (st == FL_OK) {
        a.partials = p->partials;
        a.bin_rows = rows;
        // one bucket's rows at a time, with per-tile partial sums (sized
        // above): the lagged step's per-workgroup buffers follow the plan's
        // grid, not these launches'
        a.lag = 0;
        hipError_t e = hipMemsetAsync(p->state, 0, sizeof(PrState), s);
        if (e == hipSuccess) e = fl::launch_pr_init(a, init_grid, s);
        const int64_t resident = (int64_t)std::max(per_cu, 1) * ctx->num_cus / fl::kXcds * fl::kXcds;
        int32_t begin = 0;
        for (int b = 0; b < fl::kBuckets && e == hipSuccess; ++b) {
            if (sizes[b] == 0) continue;
            int lmax = 1;
            while (lmax < 64 && lmax < bucket_hi(b)) lmax <<= 1;
            double best = -1.0;
            for (int l = 1; l <= lmax && e == hipSuccess; l <<= 1)
                for (int t = 1; t <= 4 && e == hipSuccess; t *= 4) {
                    fl::BinTable tb{};
                    tb.n_classes = 1;
                    tb.c[0].row_begin = begin;
                    tb.c[0].rows = sizes[b];
                    tb.c[0].lanes = (int16_t)l;
                    tb.c[0].blocks = (int16_t)t;
                    const int32_t per = t * (fl::kBlock / l);
                    tb.tiles = (sizes[b] + per - 1) / per;
                    const int g = (int)std::min<int64_t>(resident, (tb.tiles + fl::kXcds - 1) / fl::kXcds * fl::kXcds);
                    e = fl::launch_pr_sweep_binned(a, tb, g, s);   // warm-up
                    if (e == hipSuccess) e = hipEventRecord(p->ev[5], s);
                    for (int32_t q = 0; q < sweeps && e == hipSuccess; ++q) e = fl::launch_pr_sweep_binned(a, tb, g, s);
                    if (e == hipSuccess) e = hipEventRecord(p->ev[6], s);
                    if (e == hipSuccess) e = hipStreamSynchronize(s);
                    const double us = e == hipSuccess ? 1e3 * elapsed(p->ev[5], p->ev[6]) / sweeps : 0.0;
                    if (e == hipSuccess && (best < 0.0 || us < best)) {
                        best = us;
                        m = map_with(m, b, l, t);
                    }
                }
            begin += sizes[b];
        }
        if (e != hipSuccess) st = fail(ctx, FL_EHIP, "bucket tuning: %s", hipGetErrorString(e));
    }
    ctx->pool.release(rows);
    *map = m;
    return st;
}

}  // namespace

extern "C" {

fl_status fl_tune(fl_ctx *ctx, fl_plan *p, const fl_params *prm, int32_t sweeps, int32_t *best,
                  double *us_per_sweep) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!p || !prm || !best || p->ctx != ctx) return fail(ctx, FL_EINVAL, "bad argument");
    if (sweeps < 1 || sweeps > 1000) return fail(ctx, FL_EINVAL, "sweeps must be in [1, 1000]");
    Resolved r;
    fl_status st = resolve_params(ctx, p, prm, r);
    if (st != FL_OK) return st;
    r.tol = 0.0;                // every timed sweep does work
    r.max_iter = sweeps + 1;
    FL_HIP(hipSetDevice(ctx->device));
    FL_HIP(ensure_events(p));
    hipStream_t s = ctx->stream;
    // the bucket mapping first, so that the binned layout below is timed with it
    uint64_t map = 0;
    st = tune_buckets(ctx, p, r, sweeps, &map);
    if (st != FL_OK) return st;
    ctx->tuned_map[shape_key(p)] = map;
    const int layouts[FL_TUNE_LAYOUTS] = {FL_ROWS_SLOTS, 1, 2, 4, 8, 16, 32, 64, FL_ROWS_BINNED};
    double best_us = 0.0;
    *best = 0;
    for (int j = 0; j < FL_TUNE_LAYOUTS; ++j) {
        if (us_per_sweep) us_per_sweep[j] = -1.0;
        const int lanes = layouts[j];
        if (lanes == FL_ROWS_SLOTS && p->sl.words == 0) continue;
        PrArgs a;
        int grid = 0, init_grid = 0;
        st = prepare_pr(ctx, p, r, lanes, a, grid, init_grid);
        if (st != FL_OK) return st;
        FL_HIP(hipMemsetAsync(p->state, 0, sizeof(PrState), s));
        FL_HIP(fl::launch_pr_init(a, init_grid, s));
        // an iteration as fl_execute runs it: sweep and step kernel, or one
        // sweep with the lagged step (the warm-up sweep 0 writes its g)
        a.sweep = 0;
        FL_HIP(fl::launch_pr_iter(a, p->sp, p->sl, lanes, grid, s));  // warm-up sweep
        FL_HIP(hipEventRecord(p->ev[5], s));
        for (int32_t q = 0; q < sweeps; ++q) {
            a.sweep = q + 1;
            FL_HIP(fl::launch_pr_iter(a, p->sp, p->sl, lanes, grid, s));
        }
        FL_HIP(hipEventRecord(p->ev[6], s));
        FL_HIP(hipStreamSynchronize(s));
        const double us = 1e3 * elapsed(p->ev[5], p->ev[6]) / sweeps;
        if (us_per_sweep) us_per_sweep[j] = us;
        if (*best == 0 || us < best_us) {
            best_us = us;
            *best = lanes;
        }
    }
    ctx->tuned[shape_key(p)] = *best;
    return FL_OK;
}

fl_status fl_bucket_map(fl_ctx *ctx, const fl_plan *p, int32_t *lanes, int32_t *blocks, int64_t *rows) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!p || p->ctx != ctx) return fail(ctx, FL_EINVAL, "bad plan");
    FL_HIP(hipSetDevice(ctx->device));
    const uint64_t m = bin_map_for(ctx, shape_key(p));
    for (int b = 0; b < fl::kBuckets; ++b) {
        if (lanes) lanes[b] = map_lanes(m, b);
        if (blocks) blocks[b] = map_blocks(m, b);
    }
    if (rows) {
        int32_t *tmp = pool_alloc<int32_t>(ctx, p->n);
        if (!tmp) return fail(ctx, FL_ENOMEM, "device allocation failed");
        int32_t sizes[fl::kBuckets];
        const fl_status st = bucket_rows(ctx, p, tmp, sizes);
        ctx->pool.release(tmp);
        if (st != FL_OK) return st;
        for (int b = 0; b < fl::kBuckets; ++b) rows[b] = sizes[b];
    }
    return FL_OK;
}

// ---- batches ----

fl_status fl_batch_create(fl_ctx *ctx, fl_batch **out) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!out) return fail(ctx, FL_EINVAL, "null argument");
    *out = nullptr;
    FL_HIP(hipSetDevice(ctx->device));
    fl_batch *b = new (std::nothrow) fl_batch;
    if (!b) return fail(ctx, FL_ENOMEM, "out of host memory");
    b->ctx = ctx;
    for (int w = 0; w <= fl::kMaxWords; ++w) {
        hipError_t he = w == 0 ? fl::batch_sweep_binned_blocks_per_cu(&b->sweep_per_cu[0])
                               : fl::batch_sweep_blocks_per_cu(w, &b->sweep_per_cu[w]);
        if (he != hipSuccess) {
            delete b;
            return fail(ctx, FL_EHIP, "occupancy query: %s", hipGetErrorString(he));
        }
    }
    for (auto &e : b->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            delete b;
            return fail(ctx, FL_EHIP, "hipEventCreate failed");
        }
    }
    fl_status st = batch_reserve(b, 16, 1024);
    if (st == FL_OK && (hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess ||
                        hipStreamCreateWithFlags(&b->side_stream, hipStreamNonBlocking) != hipSuccess ||
                        hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess ||
                        hipEventCreateWithFlags(&b->join, hipEventDisableTiming) != hipSuccess)) {
        (void)hipGetLastError();
        st = fail(ctx, FL_EHIP, "stream or event creation failed");
    }
    if (st == FL_OK) {
        b->d_counts = pool_alloc<int32_t>(ctx, fl_batch::kCounts);
        if (!b->d_counts ||
            hipHostMalloc((void **)&b->h_counts, sizeof(int32_t) * fl_batch::kCounts, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            st = fail(ctx, FL_ENOMEM, "batch counters: allocation failed");
        }
    }
    if (st != FL_OK) {
        batch_free_tables(b);
        if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
        if (b->side_stream) (void)hipStreamDestroy(b->side_stream);
        if (b->fork) (void)hipEventDestroy(b->fork);
        if (b->join) (void)hipEventDestroy(b->join);
        ctx->pool.release(b->d_counts);
        for (auto &e : b->ev)
            if (e) (void)hipEventDestroy(e);
        delete b;
        return st;
    }
    *out = b;
    return FL_OK;
}

fl_status fl_batch_destroy(fl_ctx *ctx, fl_batch *b) {
    if (!ctx) return FL_EINVAL;
    if (!b) return FL_OK;
    if (b->ctx != ctx) return fail(ctx, FL_EINVAL, "batch belongs to another context");
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &m : b->members) member_release(ctx, m);
    batch_free_tables(b);
    batch_free_graphs(b);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    (void)hipStreamSynchronize(b->side_stream);
    (void)hipStreamDestroy(b->side_stream);
    (void)hipEventDestroy(b->fork);
    (void)hipEventDestroy(b->join);
    ctx->pool.release(b->d_counts);
    if (b->h_counts) (void)hipHostFree(b->h_counts);
    for (auto &e : b->ev) (void)hipEventDestroy(e);
    delete b;
    return FL_OK;
}

fl_status fl_batch_add(fl_ctx *ctx, fl_batch *b, fl_plan *p, const fl_params *prm, double *d_pagerank,
                       int32_t *d_minima, int64_t tag) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!b || !p || !prm || !d_pagerank || (!d_minima && p->m > 0)) return fail(ctx, FL_EINVAL, "null argument");
    // a plan built by another context on the same device may join (its FFG
    // is only read; the member's own buffers come from this context)
    if (b->ctx != ctx) return fail(ctx, FL_EINVAL, "batch belongs to another context");
    if (p->ctx->device != ctx->device) return fail(ctx, FL_EINVAL, "plan is on another device");
    if (prm && prm->row_mapping != 0 && !is_slot_layout(prm->row_mapping) && !is_binned_layout(prm->row_mapping))
        return fail(ctx, FL_EINVAL, "batch members run FL_ROWS_SLOTS or FL_ROWS_BINNED (0: automatic)");
    Resolved r;
    fl_status st = resolve_params(ctx, p, prm, r);
    if (st != FL_OK) return st;
    FL_HIP(hipSetDevice(ctx->device));
    // layout: the slot sweep where the space allows it and it is asked for
    // (or is the shape class's tuned layout, or nothing is tuned); else the
    // binned sweep with the plan's bins (built here, with the class's tuned
    // mapping, if the plan is this context's and has none)
    const bool slot_ok = p->sl.words > 0 && x_bytes_of(p) > 0;
    bool binned;
    if (is_slot_layout(prm->row_mapping)) {
        if (!slot_ok) return fail(ctx, FL_EINVAL, "the slot sweep cannot take a space of 2^29+ configurations");
        binned = false;
    } else if (is_binned_layout(prm->row_mapping)) {
        binned = true;
    } else {
        // a tuned lanes-per-row CSR layout wins on a lone space by spreading
        // it over more workgroups; in a batch the members supply that
        // parallelism, so such members keep the slot sweep
        const auto hit = ctx->tuned.find(shape_key(p));
        binned = !slot_ok || (hit != ctx->tuned.end() && hit->second == FL_ROWS_BINNED);
    }
    if (binned) {
        if (p->ctx == ctx) {
            st = ensure_binned(ctx, p, bin_map_for(ctx, shape_key(p)));
            if (st != FL_OK) return st;
        } else if (!p->have_bins) {
            if (!slot_ok || is_binned_layout(prm->row_mapping))
                return fail(ctx, FL_EINVAL, "the plan (of another context) has no binned rows");
            binned = false;
        }
    }
    fl_batch::Member m;
    m.plan = p;
    m.binned = binned;
    int64_t tiles = 0;
    for (const auto &q : b->members) tiles += member_tiles(q);
    st = batch_reserve(b, (int)b->members.size() + 1, tiles + member_tiles(m));
    if (st != FL_OK) return st;
    st = member_alloc(ctx, p, m);
    if (st != FL_OK) return st;
    if (binned) {
        p->bin_users += 1;
        m.holds_bins = true;
    }
    m.plan = p;
    m.prm = r;
    m.out_pr = d_pagerank;
    m.out_min = d_minima;
    m.tag = tag;
    m.slot = b->free_slots.back();
    b->free_slots.pop_back();
    fl::BatchMember &bm = b->h_members[m.slot];
    memset(&bm, 0, sizeof bm);
    bm.rec = p->rec;
    bm.presence = p->presence;
    bm.k_pad = k_pad_of(p->sl);
    bm.off = p->d_off;
    bm.valid_raw = p->valid_raw;
    bm.out_deg = p->out_deg;
    bm.minima = p->minima;
    bm.fit_c = p->fit_c;
    bm.y[0] = m.y[0];
    bm.y[1] = m.y[1];
    bm.x[0] = m.x[0];
    bm.x[1] = m.x[1];
    bm.partials = m.partials;
    bm.st = m.state;
    bm.out_pagerank = d_pagerank;
    bm.out_minima = d_minima;
    bm.d = r.d;
    bm.tol = r.tol;
    bm.threshold = (1.0 + r.p) * (double)p->f_opt;
    bm.n = (int32_t)p->n;
    bm.m = (int32_t)p->m;
    bm.k_slots = p->sl.k;
    bm.words = binned ? 0 : p->sl.words;
    bm.x_bytes = x_bytes_of(p);
    bm.n_tiles = tiles_of(p);
    bm.max_iter = r.max_iter;
    bm.xmap = binned ? nullptr : p->valid_raw;
    bm.n_parts = binned ? p->bins.tiles : tiles_of(p);
    if (binned) {
        bm.row_ptr = p->row_ptr;
        bm.col_idx = p->col_idx;
        bm.bin_rows = p->bin_rows;
        bm.bins = p->bins;
    }
    b->members.push_back(m);
    return FL_OK;
}

fl_status fl_batch_step(fl_ctx *ctx, fl_batch *b, int32_t sweeps, int32_t *n_running) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!b || b->ctx != ctx) return fail(ctx, FL_EINVAL, "bad batch");
    if (sweeps < 0) return fail(ctx, FL_EINVAL, "sweeps must be >= 0");
    FL_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const int64_t tc = b->tile_cap;
    fl::TileRef *t_init = b->h_tiles, *t_sweep = b->h_tiles + tc, *t_out = b->h_tiles + 2 * tc;
    int32_t *i_init = b->h_ids, *i_run = b->h_ids + b->capacity, *i_fin = b->h_ids + 2 * b->capacity;

    // the lists below must fit the pinned tables (each region holds tile_cap
    // tile references and capacity ids); checked before anything is written
    {
        int64_t t_join = 0, t_run = 0;
        for (const auto &m : b->members) {
            if (m.phase == 0) t_join += tiles_of(m.plan);
            if (m.phase <= 1) t_run += std::max<int64_t>(tiles_of(m.plan), m.binned ? m.plan->bins.tiles : 0);
        }
        if (t_join > tc || t_run > tc || (int64_t)b->members.size() > b->capacity)
            return fail(ctx, FL_EINVAL, "batch tables hold %lld tiles and %d members: %lld joining tiles, %lld "
                        "running tiles, %zu members", (long long)tc, b->capacity, (long long)t_join,
                        (long long)t_run, b->members.size());
    }
    // host lists: joining members and their tiles, running members and
    // their tiles grouped by record width
    int32_t n_init = 0;
    int64_t nt_init = 0;
    for (auto &m : b->members) {
        if (m.phase != 0) continue;
        i_init[n_init++] = m.slot;
        for (int32_t t = 0; t < tiles_of(m.plan); ++t) t_init[nt_init++] = {m.slot, t};
        m.phase = 1;
    }
    // running members: those the segmented launches sweep first (their ids
    // are the step kernel's list), then the small ones grouped by width
    auto small = [&](const fl_batch::Member &m) {
        return !m.binned && b->small_tiles > 0 && tiles_of(m.plan) <= b->small_tiles;
    };
    auto width = [](const fl_batch::Member &m) { return m.binned ? 0 : m.plan->sl.words; };
    int32_t n_run = 0;
    int64_t group_begin[fl::kMaxWords + 2] = {};
    int64_t nt = 0;
    for (int w = 0; w <= fl::kMaxWords; ++w) {
        group_begin[w] = nt;
        for (auto &m : b->members) {
            if (m.phase != 1 || width(m) != w || small(m)) continue;
            i_run[n_run++] = m.slot;
            const int32_t sweep_tiles = m.binned ? m.plan->bins.tiles : tiles_of(m.plan);
            for (int32_t t = 0; t < sweep_tiles; ++t) t_sweep[nt++] = {m.slot, t};
        }
    }
    group_begin[fl::kMaxWords + 1] = nt;
    int32_t small_begin[fl::kMaxWords + 2] = {};
    int32_t n_all = n_run;
    for (int w = 1; w <= fl::kMaxWords; ++w) {
        small_begin[w] = n_all;
        for (auto &m : b->members)
            if (m.phase == 1 && width(m) == w && small(m)) i_run[n_all++] = m.slot;
    }
    small_begin[fl::kMaxWords + 1] = n_all;
    int32_t *hc = b->h_counts;
    memset(hc, 0, sizeof(int32_t) * fl_batch::kCounts);
    for (int w = 0; w <= fl::kMaxWords; ++w) {
        hc[2 * w] = (int32_t)group_begin[w];
        hc[2 * w + 1] = (int32_t)(group_begin[w + 1] - group_begin[w]);
    }
    hc[fl_batch::kRunCount] = n_run;
    hc[fl_batch::kInitCount] = n_init;

    // uploads: member table (rows of members that left are never read),
    // lists, counts
    fl::TileRef *d_sweep = b->d_tiles + tc;
    int32_t *d_run = b->d_ids + b->capacity;
    FL_HIP(hipMemcpyAsync(b->d_members, b->h_members, sizeof(fl::BatchMember) * b->capacity,
                          hipMemcpyHostToDevice, s));
    FL_HIP(hipMemcpyAsync(b->d_counts, hc, sizeof(int32_t) * fl_batch::kCounts, hipMemcpyHostToDevice, s));
    if (n_init > 0) {
        FL_HIP(hipMemcpyAsync(b->d_tiles, t_init, sizeof(fl::TileRef) * nt_init, hipMemcpyHostToDevice, s));
        FL_HIP(hipMemcpyAsync(b->d_ids, i_init, sizeof(int32_t) * n_init, hipMemcpyHostToDevice, s));
        // joining members: initial iterate
        FL_HIP(fl::launch_batch_init(b->d_members, b->d_tiles, (int32_t)nt_init, b->d_ids, n_init,
                                     b->d_counts + fl_batch::kInitCount, s));
    }
    if (n_all > 0) FL_HIP(hipMemcpyAsync(d_run, i_run, sizeof(int32_t) * n_all, hipMemcpyHostToDevice, s));
    // small members: on the side stream, after the uploads and initial
    // iterates, up to 4 x sweeps each (most finish within the step)
    const bool side = n_all > n_run && sweeps > 0;
    if (side) {
        FL_HIP(hipEventRecord(b->fork, s));
        FL_HIP(hipStreamWaitEvent(b->side_stream, b->fork, 0));
        for (int w = 1; w <= fl::kMaxWords; ++w) {
            const int32_t cnt = small_begin[w + 1] - small_begin[w];
            if (cnt == 0) continue;
            FL_HIP(fl::launch_batch_small(b->d_members, d_run + small_begin[w], cnt, w, 4 * sweeps,
                                          std::min(cnt, 1024), b->side_stream));
        }
        FL_HIP(hipEventRecord(b->join, b->side_stream));
    }
    if (n_run > 0 && sweeps > 0) {
        FL_HIP(hipMemcpyAsync(d_sweep, t_sweep, sizeof(fl::TileRef) * nt, hipMemcpyHostToDevice, s));
        // launch shape: grids rounded up to powers of two (times the XCD
        // count) so that small changes of membership reuse the captured graph
        fl_batch::Shape shape;
        shape.sweeps = sweeps;
        shape.members = b->d_members;
        shape.tiles = b->d_tiles;
        shape.ids = b->d_ids;
        for (int w = 0; w <= fl::kMaxWords; ++w) {
            const int32_t cnt = hc[2 * w + 1];
            if (cnt == 0) continue;
            const int64_t resident =
                (int64_t)std::max(b->sweep_per_cu[w], 1) * ctx->num_cus / fl::kXcds * fl::kXcds;
            int64_t g = fl::kXcds;
            while (g < resident && g < cnt) g *= 2;
            shape.grid[w] = (int32_t)std::max<int64_t>(fl::kXcds, std::min(g, resident));
        }
        int32_t fg = 1;
        while (fg < n_run && fg < fl::kMaxFinishGrid) fg *= 2;
        shape.finish_grid = fg;
        auto enqueue = [&](hipStream_t q) -> hipError_t {
            for (int32_t j = 0; j < sweeps; ++j) {
                for (int w = 0; w <= fl::kMaxWords; ++w) {
                    if (shape.grid[w] == 0) continue;
                    hipError_t e = w == 0 ? fl::launch_batch_sweep_binned(b->d_members, d_sweep, b->d_counts,
                                                                          shape.grid[0], q)
                                          : fl::launch_batch_sweep(b->d_members, d_sweep, b->d_counts + 2 * w, w,
                                                                   shape.grid[w], q);
                    if (e != hipSuccess) return e;
                }
                hipError_t e = fl::launch_batch_finish(b->d_members, d_run, b->d_counts + fl_batch::kRunCount,
                                                       shape.finish_grid, q);
                if (e != hipSuccess) return e;
            }
            return hipSuccess;
        };
        // the start event goes in after any capture, so that host time spent
        // capturing is not counted as device time of the loop
        if (b->use_graphs) {
            hipGraphExec_t exec = nullptr;
            for (size_t q = 0; q < b->graphs.size(); ++q)
                if (b->graphs[q].first == shape) {
                    auto hit = b->graphs[q];   // to the most recently used end
                    b->graphs.erase(b->graphs.begin() + (long)q);
                    b->graphs.push_back(hit);
                    exec = hit.second;
                    break;
                }
            if (!exec) {
                if (b->graphs.size() >= fl_batch::kMaxGraphs) {
                    (void)hipGraphExecDestroy(b->graphs.front().second);
                    b->graphs.erase(b->graphs.begin());
                }
                // captured on the private stream (capture runs nothing),
                // launched on the context's stream
                hipGraph_t g = nullptr;
                FL_HIP(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
                const hipError_t le = enqueue(b->capture_stream);
                const hipError_t ce = hipStreamEndCapture(b->capture_stream, &g);
                if (le != hipSuccess || ce != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    return fail(ctx, FL_EHIP, "graph capture: %s",
                                hipGetErrorString(le != hipSuccess ? le : ce));
                }
                const hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (ie != hipSuccess) return fail(ctx, FL_EHIP, "graph instantiation: %s", hipGetErrorString(ie));
                b->graphs.emplace_back(shape, exec);
                ++b->graph_captures;
            }
            FL_HIP(hipEventRecord(b->ev[0], s));
            FL_HIP(hipGraphLaunch(exec, s));
            ++b->graph_launches;
        } else {
            FL_HIP(hipEventRecord(b->ev[0], s));
            FL_HIP(enqueue(s));
        }
        FL_HIP(hipEventRecord(b->ev[1], s));
        b->sweeps += sweeps;
    }
    // state of every running member
    if (side) FL_HIP(hipStreamWaitEvent(s, b->join, 0));
    if (n_all > 0) {
        FL_HIP(fl::launch_batch_states(b->d_members, d_run, n_all, b->d_states, s));
        FL_HIP(hipMemcpyAsync(b->h_states, b->d_states, sizeof(PrState) * n_all, hipMemcpyDeviceToHost, s));
    }
    FL_HIP(hipStreamSynchronize(s));
    if (n_run > 0 && sweeps > 0) b->sweep_ms += elapsed(b->ev[0], b->ev[1]);
    // members that stopped: ranks, minima, C_p
    int32_t n_fin = 0;
    int64_t nt_fin = 0;
    std::vector<int> fin_index;
    for (int32_t j = 0; j < n_all; ++j) {
        if (!b->h_states[j].done) continue;
        for (size_t q = 0; q < b->members.size(); ++q) {
            if (b->members[q].slot != i_run[j]) continue;
            fl_batch::Member &m = b->members[q];
            if (nt_fin + tiles_of(m.plan) > tc) return fail(ctx, FL_EINVAL, "batch tables: output tiles overflow");
            i_fin[n_fin++] = m.slot;
            fin_index.push_back((int)q);
            for (int32_t t = 0; t < tiles_of(m.plan); ++t) t_out[nt_fin++] = {m.slot, t};
        }
    }
    if (n_fin > 0) {
        fl::TileRef *d_out = b->d_tiles + 2 * tc;
        int32_t *d_fin = b->d_ids + 2 * b->capacity;
        FL_HIP(hipMemcpyAsync(d_out, t_out, sizeof(fl::TileRef) * nt_fin, hipMemcpyHostToDevice, s));
        FL_HIP(hipMemcpyAsync(d_fin, i_fin, sizeof(int32_t) * n_fin, hipMemcpyHostToDevice, s));
        FL_HIP(fl::launch_batch_output(b->d_members, d_out, (int32_t)nt_fin, d_fin, n_fin, b->d_states, s));
        FL_HIP(hipMemcpyAsync(b->h_states, b->d_states, sizeof(PrState) * n_fin, hipMemcpyDeviceToHost, s));
        FL_HIP(hipStreamSynchronize(s));
        for (int32_t j = 0; j < n_fin; ++j) {
            fl_batch::Member &m = b->members[fin_index[j]];
            const PrState &hs = b->h_states[j];
            fill_summary(m.plan, hs, m.binned ? FL_ROWS_BINNED : FL_ROWS_SLOTS, hs.done == 1 ? FL_OK : FL_ENOCONV,
                         &m.sum);
            m.phase = 2;
        }
    }
    if (n_running) {
        int32_t cnt = 0;
        for (const auto &m : b->members) cnt += (m.phase != 2);
        *n_running = cnt;
    }
    return FL_OK;
}

fl_status fl_batch_collect(fl_ctx *ctx, fl_batch *b, int32_t max, int64_t *tags, fl_summary *out,
                           int32_t *n_out) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!b || b->ctx != ctx || !n_out || max < 0 || (max > 0 && (!tags || !out)))
        return fail(ctx, FL_EINVAL, "bad argument");
    int32_t n = 0;
    for (size_t q = 0; q < b->members.size() && n < max;) {
        fl_batch::Member &m = b->members[q];
        if (m.phase != 2) {
            ++q;
            continue;
        }
        tags[n] = m.tag;
        out[n] = m.sum;
        ++n;
        member_release(ctx, m);   // the step that finished it synchronised the stream
        b->free_slots.push_back(m.slot);
        b->members.erase(b->members.begin() + (long)q);
    }
    *n_out = n;
    return FL_OK;
}

fl_status fl_batch_timing(fl_ctx *ctx, const fl_batch *b, int64_t *sweeps, double *sweep_ms,
                          int64_t *graph_launches, int64_t *graph_captures) {
    if (!ctx) return FL_EINVAL;
    if (!b || b->ctx != ctx) return fail(ctx, FL_EINVAL, "bad batch");
    if (sweeps) *sweeps = b->sweeps;
    if (sweep_ms) *sweep_ms = b->sweep_ms;
    if (graph_launches) *graph_launches = b->graph_launches;
    if (graph_captures) *graph_captures = b->graph_captures;
    return FL_OK;
}

fl_status fl_batch_set_small(fl_ctx *ctx, fl_batch *b, int32_t max_tiles) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!b || b->ctx != ctx) return fail(ctx, FL_EINVAL, "bad batch");
    if (max_tiles < 0 || max_tiles > 64) return fail(ctx, FL_EINVAL, "max_tiles must be in [0, 64]");
    b->small_tiles = max_tiles;
    return FL_OK;
}

fl_status fl_batch_set_graphs(fl_ctx *ctx, fl_batch *b, int32_t enable) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (!b || b->ctx != ctx) return fail(ctx, FL_EINVAL, "bad batch");
    b->use_graphs = enable != 0;
    return FL_OK;
}

fl_status fl_analyze_batch(fl_ctx *ctx, int32_t n_spaces, const fl_space *spaces, const float *const *d_fitness_raw,
                           const fl_neighbourhood *nb, const fl_params *prm, double *const *d_pagerank,
                           int32_t *const *d_minima, fl_summary *out) {
    if (!ctx) return FL_EINVAL;
    ctx->err.clear();
    if (n_spaces < 0 || (n_spaces > 0 && (!spaces || !d_fitness_raw || !nb || !prm || !d_pagerank || !d_minima || !out)))
        return fail(ctx, FL_EINVAL, "bad argument");
    FL_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    // build every FFG with one synchronisation per stage
    // Segmented build: every stage runs for all spaces in one launch (the
    // node-tile stages once per record width and buffer form) from a table of
    // per-space descriptors; the host synchronises once per stage to size the
    // next one.  Untimed builds; every build's sizes sit in one device array,
    // copied to the host in one transfer per stage.  Spaces with more than
    // kMaxSlots candidate slots launch their own generic degree and fill
    // kernels inside the same stages.
    std::vector<Build> builds((size_t)n_spaces);
    BuildSizes *h_sizes = nullptr, *d_sizes = nullptr;
    fl::SegBuild *d_segs = nullptr;
    int32_t *d_ids = nullptr;
    fl::SegTile *d_tiles = nullptr;
    if (n_spaces > 0) {
        // pinned tables (the sizes among them) kept by the context between calls
        if (seg_tables_reserve(ctx, n_spaces, 0) != FL_OK) return fail(ctx, FL_ENOMEM, "pinned allocation failed");
        h_sizes = ctx->h_seg_sizes;
        d_sizes = pool_alloc<BuildSizes>(ctx, n_spaces);
        d_segs = pool_alloc<fl::SegBuild>(ctx, n_spaces);
        d_ids = pool_alloc<int32_t>(ctx, n_spaces);
        if (!d_sizes || !d_segs || !d_ids) {
            ctx->pool.release(d_sizes);
            ctx->pool.release(d_segs);
            ctx->pool.release(d_ids);
            return fail(ctx, FL_ENOMEM, "allocation failed");
        }
    }
    fl::SegBuild *hs = ctx->h_segs;
    int32_t *hid = ctx->h_seg_ids;
    auto stage_sync = [&]() -> hipError_t {
        hipError_t e = n_spaces > 0 ? hipMemcpyAsync(h_sizes, d_sizes, sizeof(BuildSizes) * n_spaces,
                                                     hipMemcpyDeviceToHost, s)
                                    : hipSuccess;
        const hipError_t e2 = hipStreamSynchronize(s);
        return e != hipSuccess ? e : e2;
    };
    // upload the descriptor table, the id list and `nt` tiles (device tile
    // buffer regrown from the pool when needed)
    int64_t d_tile_cap = 0;
    auto upload = [&](int32_t n_ids, int64_t nt) -> hipError_t {
        if (nt > d_tile_cap) {
            ctx->pool.release(d_tiles);
            d_tiles = pool_alloc<fl::SegTile>(ctx, nt);
            d_tile_cap = d_tiles ? nt : 0;
            if (!d_tiles) return hipErrorOutOfMemory;
        }
        hipError_t e = hipMemcpyAsync(d_segs, hs, sizeof(fl::SegBuild) * n_spaces, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && n_ids > 0)
            e = hipMemcpyAsync(d_ids, hid, sizeof(int32_t) * n_ids, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && nt > 0)
            e = hipMemcpyAsync(d_tiles, ctx->h_seg_tiles, sizeof(fl::SegTile) * nt, hipMemcpyHostToDevice, s);
        return e;
    };
    auto buf_of = [](const fl_plan *p) { return 4 * p->n_raw < (int64_t(1) << 31); };
    // stage 1: compaction
    int64_t c_total = 0;
    for (int32_t j = 0; j < n_spaces; ++j) {
        Build &bd = builds[j];
        bd.timed = false;
        bd.shared_sizes = true;
        bd.defer = true;
        bd.h_sizes = h_sizes + j;
        bd.d_sizes = d_sizes + j;
        build_begin(ctx, bd, &spaces[j], d_fitness_raw[j], nb[j]);
        if (bd.status == FL_OK) c_total += (bd.p->n_raw + fl::kCompactTile - 1) / fl::kCompactTile;
    }
    hipError_t he = seg_tables_reserve(ctx, n_spaces, c_total) == FL_OK ? hipSuccess : hipErrorOutOfMemory;
    int32_t n_ids = 0;
    int64_t nt = 0;
    for (int32_t j = 0; j < n_spaces && he == hipSuccess; ++j) {
        Build &bd = builds[j];
        if (bd.status != FL_OK) continue;
        const fl_plan *p = bd.p;
        fl::SegBuild &g = hs[j];
        memset(&g, 0, sizeof g);
        g.sp = p->sp;
        g.sl = p->sl;
        g.fit = bd.fit;
        g.tile_cnt = bd.tile_cnt;
        g.tile_bad = bd.tile_bad;
        g.tile_off = bd.tile_off;
        g.tile_min = bd.tile_min;
        g.remap = bd.remap;
        g.valid_raw = p->valid_raw;
        g.fit_c = p->fit_c;
        g.sizes = bd.d_sizes;
        g.c_tiles = (int32_t)((p->n_raw + fl::kCompactTile - 1) / fl::kCompactTile);
        hid[n_ids++] = j;
        for (int32_t t = 0; t < g.c_tiles; ++t) ctx->h_seg_tiles[nt++] = {j, t};
    }
    if (he == hipSuccess) he = upload(n_ids, nt);
    if (he == hipSuccess) he = fl::launch_seg_compact(d_segs, d_tiles, (int32_t)nt, d_ids, n_ids, s);
    if (he == hipSuccess) he = stage_sync();
    // stages 2 and 3 run the slot builds grouped by (record width, buffer form)
    int64_t group_begin[fl::kMaxWords + 1][2] = {}, group_count[fl::kMaxWords + 1][2] = {};
    auto group_tiles = [&]() -> hipError_t {
        int64_t total = 0;
        for (auto &bd : builds)
            if (bd.status == FL_OK && bd.p->sl.words > 0) total += tiles_of(bd.p);
        if (seg_tables_reserve(ctx, n_spaces, total) != FL_OK) return hipErrorOutOfMemory;
        nt = 0;
        n_ids = 0;
        for (int w = 1; w <= fl::kMaxWords; ++w)
            for (int q = 0; q < 2; ++q) {
                group_begin[w][q] = nt;
                for (int32_t j = 0; j < n_spaces; ++j) {
                    const Build &bd = builds[j];
                    if (bd.status != FL_OK || bd.p->sl.words != w || (int)buf_of(bd.p) != q) continue;
                    for (int32_t t = 0; t < tiles_of(bd.p); ++t) ctx->h_seg_tiles[nt++] = {j, t};
                    hid[n_ids++] = j;
                }
                group_count[w][q] = nt - group_begin[w][q];
            }
        return hipSuccess;
    };
    // stage 2: degree count (allocations in build_degree; generic spaces launch there)
    if (he == hipSuccess) {
        for (auto &bd : builds) build_degree(ctx, bd);
        he = group_tiles();
    }
    for (int32_t j = 0; j < n_spaces && he == hipSuccess; ++j) {
        const Build &bd = builds[j];
        if (bd.status != FL_OK || bd.p->sl.words == 0) continue;
        const fl_plan *p = bd.p;
        fl::SegBuild &g = hs[j];
        g.n = (int32_t)p->n;
        g.n_tiles = tiles_of(p);
        g.in_deg = bd.in_deg;
        g.out_deg = p->out_deg;
        g.rec = p->rec;
        g.presence = p->presence;
        g.off_table = p->d_off;
        g.k_pad = k_pad_of(p->sl);
        g.tile_e = bd.tile_e;
        g.tile_eoff = bd.tile_eoff;
        g.tile_m = bd.tile_m;
        g.tile_moff = bd.tile_moff;
        g.fit_bytes = buf_of(p) ? (int32_t)(4 * p->n_raw) : 0;
        g.remap_bytes = g.fit_bytes;
    }
    if (he == hipSuccess) he = upload(n_ids, nt);
    for (int w = 1; w <= fl::kMaxWords && he == hipSuccess; ++w)
        for (int q = 0; q < 2 && he == hipSuccess; ++q)
            if (group_count[w][q] > 0)
                he = fl::launch_seg_degree(d_segs, d_tiles + group_begin[w][q], (int32_t)group_count[w][q], w,
                                           q != 0, s);
    if (he == hipSuccess) he = fl::launch_seg_degree_scan(d_segs, d_ids, n_ids, s);
    if (he == hipSuccess) he = stage_sync();
    // stage 3: CSR fill (col_idx allocated in build_fill; generic spaces launch there)
    if (he == hipSuccess) {
        for (auto &bd : builds) build_fill(ctx, bd);
        he = group_tiles();
    }
    for (int32_t j = 0; j < n_spaces && he == hipSuccess; ++j) {
        const Build &bd = builds[j];
        if (bd.status != FL_OK || bd.p->sl.words == 0) continue;
        const fl_plan *p = bd.p;
        fl::SegBuild &g = hs[j];
        g.n_edges = (int32_t)p->e;
        g.row_ptr = p->row_ptr;
        g.col_idx = p->col_idx;
        g.minima = p->minima;
    }
    if (he == hipSuccess) he = upload(n_ids, nt);
    for (int w = 1; w <= fl::kMaxWords && he == hipSuccess; ++w)
        for (int q = 0; q < 2 && he == hipSuccess; ++q)
            if (group_count[w][q] > 0)
                he = fl::launch_seg_fill(d_segs, d_tiles + group_begin[w][q], (int32_t)group_count[w][q], w,
                                         q != 0, s);
    const hipError_t hf = hipStreamSynchronize(s);
    if (he == hipSuccess) he = hf;
    for (auto &bd : builds) {
        if (he != hipSuccess && bd.status == FL_OK) build_fail(bd, FL_EHIP, "%s", hipGetErrorString(he));
        build_end(ctx, bd);
    }
    ctx->pool.release(d_sizes);
    ctx->pool.release(d_segs);
    ctx->pool.release(d_ids);
    ctx->pool.release(d_tiles);
    fl_status worst = FL_OK;
    std::vector<fl_status> status((size_t)n_spaces, FL_OK);
    // PageRank: batchable spaces together, the others one at a time
    // (the context keeps one batch for this between calls: its tables and
    // captured graph are reused; it is empty between calls)
    fl_status st = FL_OK;
    if (!ctx->analyze_batch) st = fl_batch_create(ctx, &ctx->analyze_batch);
    if (st != FL_OK) {
        ctx->analyze_batch = nullptr;
        for (auto &bd : builds) build_abort(ctx, bd);
        return st;
    }
    fl_batch *b = ctx->analyze_batch;
    {
        // room for every space that may join, reserved once
        int32_t cap = 0;
        int64_t tiles = 0;
        for (auto &bd : builds)
            if (bd.status == FL_OK) {
                ++cap;
                tiles += tiles_of(bd.p);
            }
        if (cap > 0) st = batch_reserve(b, (int)b->members.size() + cap, tiles);
        if (st != FL_OK) {
            for (auto &bd : builds) build_abort(ctx, bd);
            return st;
        }
    }
    int32_t in_batch = 0;
    for (int32_t j = 0; j < n_spaces; ++j) {
        memset(&out[j], 0, sizeof out[j]);
        Build &bd = builds[j];
        if (bd.status != FL_OK) {
            status[j] = bd.status;
            out[j].status = bd.status;
            continue;
        }
        fl_plan *p = bd.p;
        Resolved r;
        if (resolve_params(ctx, p, &prm[j], r) != FL_OK) {
            status[j] = FL_EINVAL;
            out[j].status = FL_EINVAL;
            fill_sizes(p, &out[j]);
            out[j].status = FL_EINVAL;
            continue;
        }
        // every space joins the batch (slot or binned sweep); an explicit
        // lanes-per-row CSR layout runs alone
        const int32_t rm = prm[j].row_mapping;
        if (rm == 0 || is_slot_layout(rm) || is_binned_layout(rm)) {
            st = fl_batch_add(ctx, b, p, &prm[j], d_pagerank[j], d_minima[j], j);
            if (st == FL_OK) {
                ++in_batch;
                continue;
            }
            if (st == FL_EHIP) break;
        }
        st = fl_execute(ctx, p, &prm[j], d_pagerank[j], d_minima[j], &out[j]);
        status[j] = st;
    }
    int32_t running = in_batch;
    while (running > 0 && st != FL_EHIP) {
        st = fl_batch_step(ctx, b, 16, &running);   // 16 sweeps per host round trip
        if (st != FL_OK) break;
        int64_t tags[64];
        fl_summary sums[64];
        int32_t got = 0;
        do {
            fl_batch_collect(ctx, b, 64, tags, sums, &got);
            for (int32_t q = 0; q < got; ++q) {
                out[tags[q]] = sums[q];
                status[tags[q]] = (fl_status)sums[q].status;
            }
        } while (got == 64);
    }
    const std::string msg = ctx->err;
    if (st != FL_OK || !b->members.empty()) {   // not drained: start afresh next time
        fl_batch_destroy(ctx, b);
        ctx->analyze_batch = nullptr;
    }
    // one synchronisation for all the call's plans
    (void)hipStreamSynchronize(s);
    for (auto &bd : builds)
        if (bd.p) plan_free(bd.p);
    ctx->err = msg;
    if (st != FL_OK) return st;
    for (int32_t j = 0; j < n_spaces; ++j)
        if (status[j] != FL_OK && (worst == FL_OK || worst == FL_ENOCONV)) worst = status[j];
    if (worst != FL_OK && ctx->err.empty()) ctx->err = "at least one space failed; see the per-space status";
    return worst;
}

}  // extern "C"
