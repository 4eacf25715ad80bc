// fl_internal.h - types shared by the engine (fl_engine.hip) and the gfx950
// kernels (fl_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fl {

constexpr int kMaxParams = 32;
constexpr int kMaxSlots = 256;                    // candidate slots a node record can hold
constexpr int kMaxWords = 5;                      // 64-bit words per node record
constexpr int kBlock = 256;                       // threads per workgroup (4 waves of 64)
constexpr int kCompactItems = 8;                  // raw configurations per thread in compaction
constexpr int kCompactTile = kBlock * kCompactItems;
// single-pass compaction of one space: 16 per thread, 4096 per tile (about
// 1 100 tiles at 4.7 M configurations, all resident at once with 32 KB of
// LDS staging each)
constexpr int kSingleItems = 16;
constexpr int kSingleTile = kBlock * kSingleItems;
constexpr int kXcds = 8;                          // MI355X: 8 XCDs, workgroups dealt round-robin
constexpr int kBatch = 16;                        // candidate slots whose loads are issued together
constexpr int kMaxFinishGrid = 1024;              // workgroups of the batched step kernel (grid-stride)
constexpr int kFinishBlock = 1024;                // threads of a step kernel workgroup (1 mod 3)
constexpr int kFillStage = 6144;                  // col_idx entries of a tile assembled in LDS by the fill
constexpr int kSmallTiles = 16;                   // batch members of at most this many tiles iterate in one workgroup

// Mixed-radix description of a search space X = S_1 x ... x S_n, parameter 0
// most significant: stride[i] = prod_{j>i} radix[j].  Digits are peeled off
// from the least significant end with q / radix = (q * magic) >> shift, exact
// for every q < 2^31 (Granlund-Montgomery with a 33-bit multiplier).
struct SpaceDesc {
    int32_t n;
    int32_t n_raw;
    int32_t radix[kMaxParams];
    int32_t stride[kMaxParams];
    uint64_t magic[kMaxParams];
    uint32_t shift[kMaxParams];
};

// Candidate neighbour slots, numbered independently of the node: slot s moves
// parameter dim[s] by delta[s] list positions, i.e. to raw index i + off[s]
// with off[s] = delta[s] * stride[dim[s]].  Hamming (eq. 2) gives parameter k
// the 2(radix_k - 1) deltas +-1 .. +-(radix_k - 1); adjacent gives +-1.  A
// slot exists for a node iff 0 <= x_k + delta < radix_k.  Slots are sorted by
// off, so ascending slot order is ascending neighbour raw index (= node id).
//
// Node record (words x 64 bits): bits [0, k) flag the slots that are in-edges
// of the node; in the last word, bits 24..31 hold out_deg and bits 32..63 the
// raw index.  words = 0 when k + 40 > 64 * kMaxWords (then only the generic
// kernels and the CSR sweep are used).
struct SlotTable {
    int32_t k;
    int32_t words;
    int32_t off[kMaxSlots];
    int16_t delta[kMaxSlots];
    uint8_t dim[kMaxSlots];
    // Parameter k's slots form two contiguous runs in slot order (every
    // offset of a less significant parameter is below the stride of a more
    // significant one): deltas -len..-1 at [neg[k], neg[k] + len[k]) and
    // +1..+len at [pos[k], pos[k] + len[k]).
    int16_t blk_neg[kMaxParams], blk_pos[kMaxParams], blk_len[kMaxParams];
};

// Sizes produced on the device by the build scans, copied to the host once.
struct BuildSizes {
    int32_t n_valid;
    int32_t n_bad;       // fitness <= 0 or -inf
    float f_opt;         // minimum valid fitness
    int32_t n_minima;
    int64_t n_edges;
    int32_t n_plateau;   // minima with a neighbour of equal fitness
    int32_t pad;
};

// One space of a segmented build: every space of a batch runs each build
// stage in the same launch (the node-tile stages once per record width and
// buffer form), each workgroup finding its space and tile in a tile list.
// Fields are filled stage by stage as the sizes become known on the host.
struct SegBuild {
    SpaceDesc sp;
    SlotTable sl;
    const float *fit;
    // compaction (sizes known from n_raw)
    int32_t *tile_cnt, *tile_bad, *tile_off;
    float *tile_min;
    int32_t *remap, *valid_raw;
    float *fit_c;
    BuildSizes *sizes;
    // degree pass (after the compaction: N)
    int32_t *in_deg, *out_deg;
    uint64_t *rec, *presence;
    int32_t *off_table;
    int64_t *tile_e, *tile_eoff;
    int32_t *tile_m, *tile_moff;
    // CSR fill (after the degree pass: E)
    int32_t *row_ptr, *col_idx, *minima;
    int32_t c_tiles, n_tiles, n, n_edges, k_pad, fit_bytes, remap_bytes, pad;
};
struct SegTile {
    int32_t seg, tile;
};


// Power-iteration state, device resident.  The stored iterate y_k is the
// normalised rank vector up to the factor s = 1/sum(y_k).
struct PrState {
    int32_t k;           // iterations completed
    int32_t done;        // 0 running, 1 converged, 2 iteration cap reached
    uint32_t ticket;     // last-workgroup election, reset by the elected one
    int32_t worked;      // iteration launches that did work
    double s;            // 1 / sum(y_k)
    double c;            // d*(sink mass)/N + (1-d)/N for the next iteration
    double sigma;        // sum(y_k)
    double resid;        // ||r_k - r_{k-1}||_1
    double resid_prev;
    double sink;         // sum of y_k over sinks
    double score_num;    // sum of ranks over L_p
    double score_den;    // sum of ranks over L
    // Lagged step (PrArgs::lag): sweep j adds the teleport-and-sink term of
    // r_{j-1}, gam[j & 1][0], and the residual of r_j against r_{j-1} uses
    // gam[j & 1][1] as well (the term of r_{j-2}); the result is the iterate
    // r = w + out_gamma in y buffer out_buf, whose entries sum to out_sigma.
    double gam[2][2];
    double out_gamma;
    double out_sigma;
    int32_t out_buf;
    int32_t lag_pad;
};

// Row formats of the PageRank sweep.
enum SweepKind : int32_t {
    kSweepCsr = 0,    // pull over the CSR, L lanes per row, x indexed by node id
    kSweepSlots = 1,  // pull over the records' in-edge slot bits, x indexed by raw index
    kSweepBinned = 2  // pull over the CSR with rows binned by in-degree, each bin its own lanes per row
};

// Rows binned by in-degree: bucket 0 holds in-degree 0, bucket b >= 1 the
// in-degrees [2^(b-1), 2^b), the last bucket everything above.  A mapping
// gives every bucket its lanes per row L and rows blocks per tile T; buckets
// with the same (L, T) form one class, whose rows (node ids, ascending) are
// contiguous in the plan's bin_rows array.  A tile of a class is T blocks of
// kBlock / L rows and writes one partial-sum triple.
constexpr int kBuckets = 8;
struct BinClass {
    int32_t row_begin;   // first entry of the class in bin_rows
    int32_t rows;
    int32_t tile_begin;  // index of its first tile (and partial triple)
    int16_t lanes;       // L
    int16_t blocks;      // T
};
struct BinTable {
    int32_t n_classes;
    int32_t tiles;       // total tiles = partial triples of a sweep
    BinClass c[kBuckets];
};
__host__ __device__ inline int bucket_of(int32_t deg) {
    if (deg <= 0) return 0;
    int b = 1;
    while (b < kBuckets - 1 && deg >= (1 << b)) ++b;
    return b;
}

struct PrArgs {
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const int32_t *out_deg;
    const int32_t *valid_raw;
    const uint64_t *rec;    // node records (SlotTable), slot sweep only
    const uint64_t *presence;  // per wave of 64 nodes: OR of their in-edge slot bits
    const int32_t *off;     // 2 k_pad entries: slot raw-index offsets (SlotTable.off, 0 past k_slots),
                            // then the byte offsets 4 (off[s] - off[0]) of the buffer-load sweep
    int32_t k_slots;
    int32_t k_pad;          // stride of off's two halves: k_slots rounded up to 64, plus 64
    float *y[3];            // iterate (node ids): y[k & 1] holds y_k; lagged step: y[j % 3] holds w_j
    float *x[2];            // y / out_deg (0 at sinks): node ids (CSR) or raw indices (slots)
    double *partials;       // 3 doubles per tile (slot sweep) or per workgroup (CSR sweep)
    PrState *st;
    int32_t n;              // N
    int32_t kind;           // SweepKind
    double d;               // damping
    double tol;
    int32_t max_iter;
    int32_t adjacent;
    int32_t x_bytes;        // slot sweep: bytes its buffer loads span (x from the most negative slot
                            // offset to the end plus the largest), when < 2^31; else 0 (plain loads)
    int32_t exact;          // 1: Jacobi sweeps u <- 1 + d P u to an exact fixed point (s = c = 1)
    const int32_t *bin_rows;  // binned sweep: node ids grouped by class
    BinTable bins;            // binned sweep: classes and tiles
    // Lagged step (lag != 0): the sweeps run back to back with no step
    // kernel.  Sweep j (the host passes j in `sweep`) writes one partial
    // triple per workgroup, as three arrays of part_stride doubles, to
    // buffer j & 1 of `partials`; its workgroup 0 first reduces the n_parts
    // triples sweep j - 1 wrote into the state that sweep j + 1 reads.
    // The stored iterate w_j leaves out the constant teleport-and-sink term
    // gamma_{j-1} of r_j = w_j + gamma_{j-1}, which only the next step
    // knows; g (node ids) holds the in-edge sums of the first sweep, whose
    // x is r_0 / out_deg with r_0 = y0 = 1/N everywhere, so g / y0 is
    // P^T D^-1 1 and gamma_{j-1} g / y0 is what the constant contributes to
    // the next edge sums.
    int32_t lag;
    int32_t sweep;
    int32_t n_parts;
    int32_t part_stride;
    int64_t n_sinks;
    float *g;
};

// One member of a batch: an FFG with its own power iteration, run together
// with the other members in segmented launches.  Device resident.
struct BatchMember {
    const uint64_t *rec;       // node records
    const uint64_t *presence;  // per-wave slot presence
    const int32_t *off;        // 2 k_pad entries, as in PrArgs
    const int32_t *valid_raw;
    const int32_t *out_deg;
    const int32_t *minima;
    const float *fit_c;
    float *y[2];
    float *x[2];               // raw-index space
    double *partials;          // 3 per tile: sum y, residual, sink sum
    PrState *st;
    double *out_pagerank;      // caller's outputs
    int32_t *out_minima;
    double d, tol, threshold;
    int32_t n, m, k_slots, k_pad, words, x_bytes, n_tiles, max_iter;
    // binned members (words == 0 in the batch's lists): CSR, bin rows and
    // classes; x indexed by node id; a sweep writes bins.tiles partial
    // triples (the initial iterate n_tiles, one per kBlock nodes)
    const int32_t *row_ptr, *col_idx, *bin_rows;
    const int32_t *xmap;       // node -> x index for the initial iterate (valid_raw, or null for node ids)
    int32_t n_parts;           // partial triples a sweep writes
    int32_t pad;
    BinTable bins;
};

struct TileRef {
    int32_t member;  // index into the member table
    int32_t tile;    // tile of that member (kBlock nodes)
};

// ---- launchers (fl_kernels.hip); all enqueue on `stream` ----
// Compaction of one space (two passes, no scan kernel): tile_cnt,
// tile_min and tile_bad hold ceil(n_raw / kSingleTile) entries.
hipError_t launch_compact_single(const float *fit, int32_t n_raw, int32_t *tile_cnt, float *tile_min,
                                 int32_t *tile_bad, int32_t *remap, int32_t *valid_raw, float *fit_c,
                                 BuildSizes *sizes, hipStream_t stream);
// Segmented build stages (see SegBuild): `tiles` lists (space, tile) pairs,
// `ids` the spaces of the one-workgroup-per-space scans.
hipError_t launch_seg_compact(const SegBuild *segs, const SegTile *tiles, int32_t n_tiles, const int32_t *ids,
                              int32_t n_ids, hipStream_t stream);
hipError_t launch_seg_degree(const SegBuild *segs, const SegTile *tiles, int32_t n_tiles, int words, bool buf,
                             hipStream_t stream);
hipError_t launch_seg_degree_scan(const SegBuild *segs, const int32_t *ids, int32_t n_ids, hipStream_t stream);
hipError_t launch_seg_fill(const SegBuild *segs, const SegTile *tiles, int32_t n_tiles, int words, bool buf,
                           hipStream_t stream);
hipError_t launch_degree(const SpaceDesc &sp, const SlotTable &sl, int adjacent, const float *fit,
                         const int32_t *valid_raw, int32_t n, int32_t *in_deg, int32_t *out_deg,
                         uint64_t *rec, uint64_t *presence, int32_t *off_table, int32_t k_pad,
                         int64_t *tile_e, int32_t *tile_m, int64_t *tile_eoff, int32_t *tile_moff,
                         BuildSizes *sizes, hipStream_t stream);
hipError_t launch_fill(const SpaceDesc &sp, const SlotTable &sl, int adjacent, const float *fit,
                       const int32_t *valid_raw, const int32_t *remap, const uint64_t *rec,
                       const uint64_t *presence, int32_t n, int32_t n_edges, const int32_t *in_deg,
                       const int32_t *out_deg, const int64_t *tile_eoff, const int32_t *tile_moff,
                       int32_t *row_ptr, int32_t *col_idx, int32_t *minima, hipStream_t stream);
hipError_t launch_pr_init(const PrArgs &a, int grid, hipStream_t stream);
hipError_t launch_pr_iter(const PrArgs &a, const SpaceDesc &sp, const SlotTable &sl, int lanes,
                          int grid, hipStream_t stream);
// The two halves of launch_pr_iter: the sweep kernel, then the step kernel.
hipError_t launch_pr_sweep(const PrArgs &a, const SlotTable &sl, int lanes, int grid, hipStream_t stream);
hipError_t launch_pr_step(const PrArgs &a, int grid, hipStream_t stream);
// Workgroups of the sweep kernel for this layout that fit on one CU at once.
hipError_t pr_iter_blocks_per_cu(const PrArgs &a, const SpaceDesc &sp, const SlotTable &sl, int lanes,
                                 int *blocks);
hipError_t launch_pr_output(const PrArgs &a, double *pagerank, hipStream_t stream);
// Binning of the rows by in-degree class: class_of[b] is the class of bucket
// b.  Count per (class, node tile) into cnt (kBuckets x n_tiles, class-major),
// scan it into off and totals (kBuckets entries), write bin_rows.
hipError_t launch_bin_rows(const int32_t *row_ptr, int32_t n, const int8_t *class_of_dev, int32_t *cnt,
                           int32_t *off, int32_t *totals, int32_t *bin_rows, hipStream_t stream);
// One binned sweep restricted to the given table (the autotuner times one
// class at a time this way), without the step kernel.
hipError_t launch_pr_sweep_binned(const PrArgs &a, const BinTable &t, int grid, hipStream_t stream);
hipError_t pr_binned_blocks_per_cu(int *blocks, bool lag = false);
hipError_t launch_batch_sweep_binned(const BatchMember *members, const TileRef *tiles, const int32_t *range_dev,
                                     int grid, hipStream_t stream);
hipError_t batch_sweep_binned_blocks_per_cu(int *blocks);
hipError_t launch_score(const double *pagerank, const int32_t *minima, int32_t m,
                        const float *fit_c, double threshold, PrState *st, hipStream_t stream);
// C_p for n thresholds: num[j], den[j] = rank sums over minima below
// thresholds[j] and over all minima (one workgroup per threshold).
hipError_t launch_score_curve(const double *pagerank, const int32_t *minima, int32_t m, const float *fit_c,
                              const double *thresholds, int32_t n, double *num_den, hipStream_t stream);
// f_opt / f(m) for every minimum, and a histogram of it over n_bins equal
// bins of [0, 1] (hist zeroed here).
hipError_t launch_naive(const int32_t *minima, int32_t m, const float *fit_c, float f_opt, double *ratio,
                        int32_t n_bins, uint32_t *hist, hipStream_t stream);

// Batched power iteration.  `tiles` lists the tiles to work on; `members`
// lists member indices for the per-member kernels.  The sweep kernel reads
// its list's start and length (range_dev[0], range_dev[1]) and the step
// kernel its list length from device memory, so launches captured in a
// graph stay valid while the lists change between replays.
hipError_t launch_batch_init(const BatchMember *members, const TileRef *tiles, int32_t n_tiles,
                             const int32_t *member_ids, int32_t n_members, const int32_t *n_members_dev,
                             hipStream_t stream);
hipError_t launch_batch_sweep(const BatchMember *members, const TileRef *tiles, const int32_t *range_dev,
                              int words, int grid, hipStream_t stream);
hipError_t batch_sweep_blocks_per_cu(int words, int *blocks);
hipError_t launch_batch_finish(const BatchMember *members, const int32_t *member_ids, const int32_t *n_members_dev,
                               int grid, hipStream_t stream);
// Small members of record width `words`, one workgroup each (grid-stride):
// up to max_sweeps sweeps and steps per member, back to back in the
// workgroup, until it stops.
hipError_t launch_batch_small(const BatchMember *members, const int32_t *member_ids, int32_t n_members, int words,
                              int32_t max_sweeps, int grid, hipStream_t stream);
hipError_t launch_batch_output(const BatchMember *members, const TileRef *tiles, int32_t n_tiles,
                               const int32_t *member_ids, int32_t n_members, PrState *states_out,
                               hipStream_t stream);
hipError_t launch_batch_states(const BatchMember *members, const int32_t *member_ids, int32_t n_members,
                               PrState *states_out, hipStream_t stream);

}  // namespace fl
