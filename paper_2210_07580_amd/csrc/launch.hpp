// Host-side launchers of the pipeline phases, shared between the
// translation units.  Every launcher takes plain device pointers and a
// stream and returns the launch status.
//
// A call clusters a batch of independent instances (a plain dbscan() call is
// a batch of one).  Points of instance k occupy the global index range
// [off_k, off_k + n_k); the packed grid identifier carries k in its top
// field, so the single stable sort keeps every instance's points in that
// same range, grids never mix instances, and each grid finds its instance's
// eps, MinPts and d through the table below.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gritdbscan.h"

namespace gd {

// Type a kernel compares squared distances with eps^2 in: 32 bits for eps
// <= GD_EPS_MAX, 64 bits above (the wide path).
template <bool kWide>
struct Dist {
    using T = uint32_t;
};
template <>
struct Dist<true> {
    using T = uint64_t;
};

constexpr int kMaxD = 8;
constexpr int kMaxLevels = kMaxD + 1;  // grid tree: instance level + one level per dimension
constexpr int kPointTile = 4096;       // default points per workgroup in the point-indexed kernels
constexpr int kMaxKeyBits = 128;       // packed grid identifiers: one word (<= 64 bits) or two

// Error bits raised by kernels into the device error word.
enum : uint32_t {
    kErrNotInteger = 1u,    // a coordinate is not a finite integer of magnitude <= 2^24
    kErrMergeRunaway = 2u,  // FastMerging exceeded its iteration bound (cannot happen; checked anyway)
    kErrKeyBits = 4u,       // packed identifiers need more than kMaxKeyBits bits
    kErrNeiOverflow = 8u,   // neighbour lists exceed the buffer given to a sync-free run
    kErrCoreCap = 16u,      // a grid's core set exceeds the merge step's LDS bitmap
    kErrPlan = 32u,         // a sync-free run met more data than it was planned for (or bad input)
};

// One clustering instance.  The host fills the first part; the layout
// kernel fills the identifier layout from the data.
struct Inst {
    const float* x;    // DEVICE, n x d row-major
    int32_t* labels;   // DEVICE out, n
    uint8_t* core;     // DEVICE out, n
    int64_t off;       // first global point index
    int64_t n;
    int64_t eps;
    int32_t d;
    int32_t minpts;
    uint32_t T;        // eps^2 (eps <= GD_EPS_MAX)
    uint32_t Tm;       // (eps + delta)^2: FastMerging's "yes" bound (delta 0: exact)
    uint64_t T64;      // eps^2 and (eps + delta)^2 in 64 bits: the wide path, for any eps
    uint64_t Tm64;
    uint32_t tile0;    // first point tile of the instance (tiles never straddle instances)
    // filled on the device
    int32_t mn[kMaxD];
    int32_t mx[kMaxD];
    int32_t bits[kMaxD];
    int32_t shift[kMaxD];
    int32_t key_bits;
    uint32_t err;
};

// eps^2 and FastMerging's "yes" bound in the width a kernel compares in.
template <bool kWide>
__device__ __forceinline__ typename Dist<kWide>::T inst_T(const Inst& I) {
    if constexpr (kWide) return I.T64; else return I.T;
}
template <bool kWide>
__device__ __forceinline__ typename Dist<kWide>::T inst_Tm(const Inst& I) {
    if constexpr (kWide) return I.Tm64; else return I.Tm;
}

// Batch-wide identifier layout and counters (device).
struct Header {
    int32_t inst_shift;   // position of the instance field (max over instances of key_bits)
    int32_t total_bits;   // bits of the packed identifier
    uint32_t err;         // OR of all error bits
    uint32_t ncell;       // |Gs| over the batch
    uint32_t level_count[kMaxLevels];
    uint32_t counts[5];   // core points, core grids, max core points per grid, dense grids, tiny core grids
    uint32_t pad;
    uint64_t nei_total;
};

struct Batch {
    const Inst* inst;     // device table
    int32_t count;
    int32_t D;            // largest d in the batch (coordinate rows; shorter points are padded with 0)
    int64_t n;            // total points
    uint32_t tiles;       // point tiles over the batch
    uint32_t tile_pts;    // points per tile (a multiple of 256): one workgroup each
    Header* hdr;          // device
};

// Instance of point tile `tile` (uniform per workgroup): the last k with tile0 <= tile.
__device__ __forceinline__ int tile_instance(const Batch& b, uint32_t tile) {
    int lo = 0, hi = b.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.inst[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Grid tree (Section 4.2.1) as flat level arrays.  Level 0 holds one node
// per instance present; level l >= 1 holds one node per distinct prefix
// (instance, g_1, ..., g_l), in lexicographic order; key[l][a] is the node's
// identifier in dimension l (the instance id at level 0).  For l < L-1 the
// children of node a are the level-(l+1) nodes [child[l][a], child[l][a+1]);
// the nodes of the last level are the grids themselves.
struct TreeView {
    const int32_t* key[kMaxLevels];
    const uint32_t* child[kMaxLevels];
    const uint32_t* level_count;  // device: nodes per level
};

// Sorted points and grids.
struct GridView {
    Batch b;
    int64_t n;                   // total points
    int D;                       // coordinates per row (shorter points padded with 0)
    const int32_t* crd;          // rows of row_stride(D) int32: coordinates minus the instance minimum,
                                 // sorted by grid (row s = sorted point s)
    const uint32_t* sidx;        // n: global input index of each sorted point
    int64_t ncell;               // grids (exact, or an upper bound when the launch is sync-free)
    const uint32_t* ncell_dev;   // device: exact number of grids
    const uint32_t* cell_start;  // ncell + 1
    const int32_t* ck;           // (D + 1) x ck_stride: row 0 instance id, rows 1..D identifiers
    int64_t ck_stride;
};

// The instance of grid c (a single-instance call skips the identifier load).
__device__ __forceinline__ const Inst& cell_inst(const GridView& g, int64_t c) {
    return g.b.inst[g.b.count == 1 ? 0 : g.ck[c]];
}

// ---- partition.hip
// Minima and maxima of every instance, then the identifier layout.  part:
// scratch of 2 * kMaxD int32 per point tile; plan_bits: identifier bits a
// sync-free run sorts (64 otherwise); more raise kErrPlan.
hipError_t launch_minmax(const Batch& b, int32_t* part, int plan_bits, hipStream_t st);
// Sync-free runs: compare the device counts with the capacities the run was
// planned with (stage 0: grids; 1: neighbour entries; 2: core grids and the
// largest core set).  On overflow, or after an input error, kErrPlan goes up
// and the grid count drops to zero, so every later kernel finds no work.
hipError_t launch_plan_check(Header* hdr, int stage, int64_t cap_a, int64_t cap_b, hipStream_t st);
// Packed rows: each coordinate's low pack_bits(d) bits ride through the sort
// in the high half of a 64-bit value (the point's index in the low half).
// The grid's centre recovers the rest when it lies within 2^(bits-1) of
// every coordinate of the grid: eps / sqrt(d) + 4 < 2^bits (with margin).
__host__ __device__ constexpr int pack_bits(int d) { return 32 / d; }
__host__ __device__ inline bool pack_fits(int d, int64_t eps) {
    return d >= 1 && d <= kMaxD && (double)eps / sqrt((double)d) + 4.0 < (double)(1ull << pack_bits(d));
}
// Packed rows with two-word keys: identifiers wider than 32 bits carry the
// low bits of the coordinates in the same 64-bit sort word, below the
// identifier: word = identifier << (D * B) | sum_j (u_j mod 2^B) << (j * B),
// with one width B for the whole batch, and the sort orders on the
// identifier bits alone.  pack64_bits(d, eps): the smallest B that holds a
// grid of instance (d, eps), by the same bound as pack_fits; 0 if none up to
// 31 does.
__host__ __device__ inline bool pack_fits_bits(int d, int64_t eps, int bits) {
    return d >= 1 && d <= kMaxD && bits >= 1 && bits <= 31 &&
           (double)eps / sqrt((double)d) + 4.0 < (double)(1ull << bits);
}
inline int pack64_bits(int d, int64_t eps) {
    for (int bits = 1; bits <= 31; ++bits)
        if (pack_fits_bits(d, eps, bits)) return bits;
    return 0;
}
// The words of the batch in input order (B bits per coordinate of the
// batch's D).  A sync-free run whose instance table no longer fits B raises
// kErrPlan.
hipError_t launch_keys_packed64(const Batch& b, uint64_t* words, int bits, hipStream_t st);
// After the sort: each sorted word becomes its identifier again (in place)
// and the sorted rows are rebuilt from it (crd as for launch_unpack).
hipError_t launch_unpack64(const Batch& b, uint64_t* words, int bits, int32_t* crd, hipStream_t st);
// Grid identifiers in input order; with vals (n entries), also the packed
// sort values (index | low coordinate bits << 32).
template <typename K>
hipError_t launch_keys(const Batch& b, K* keys, uint64_t* vals, hipStream_t st);
// Sorted point rows: crd row s = point sidx[s] (see GridView::crd).
hipError_t launch_gather(const Batch& b, const uint32_t* sidx, int32_t* crd, hipStream_t st);
// The same rows, and sidx, from the sorted identifiers and packed values
// (32-bit identifiers; every instance pack_fits).
hipError_t launch_unpack(const Batch& b, const uint32_t* skeys, const uint64_t* vals, uint32_t* sidx, int32_t* crd,
                         hipStream_t st);
// Runs of equal keys: cell_start[0..ncell], identifiers; header ncell written.
template <typename K>
hipError_t launch_cells(const Batch& b, const K* skeys, uint32_t* partial, uint32_t* cell_start,
                        int32_t* ck, int64_t ck_stride, hipStream_t st);
// Grid tree levels over the sorted grids.  level_excl: D x (ncell+1) scratch;
// partial: scan scratch of 64-bit words (passed as the u32 view).
hipError_t launch_tree(const GridView& g, uint32_t* level_excl, uint32_t* partial, int32_t* const* tkey,
                       uint32_t* const* tchild, hipStream_t st);

// ---- neighbors.hip (Algorithm 3)
// The query that produces the lists: the grid tree with offset-ordered lists
// (walk order above 2^20 grids), the grid tree in walk order always, or
// direct hashing of every candidate identifier (offset-ordered).
enum NeiQueryKind { kNeiTree = 0, kNeiTreeWalkOrder = 1, kNeiHash = 2 };
// Option value of GD_OPT_NEIGHBOR_QUERY 0: the tree in offset order or walk
// order by the grids' mean size (resolved on the host per call).
constexpr int kNeiAuto = 3;
struct NeiQuery {
    TreeView t;
    int kind;
    // hashing only: the identifier -> grid table (launch_grid_table)
    const void* table;
    int bits;
    int key_bytes;          // 4 or 8
    const Inst* inst;       // device instance table
    const int* inst_shift;  // device: Header::inst_shift
};
// Pass 1: per-grid neighbour count per offset value (ncell x D, u32).
// lane_cnt (optional, nei_lane_count_words u32; nullptr when that is 0 or
// no room): the split query's per-lane counts, kept for pass 2.
// only_big (optional): per-grid core counts; then only grids with more than
// kTinyCore core points get a list, the others an empty one.
int64_t nei_lane_count_words(const NeiQuery& nq, int64_t ncell, int D);
// Whether the lists of this query come out in walk order (then the fill
// also writes each list's larger-index range, nei_up).
bool nei_walk_order(const NeiQuery& nq, int64_t ncell);
hipError_t launch_nei_count(const GridView& g, const NeiQuery& nq, uint32_t* off_counts, uint32_t* lane_cnt,
                            const uint32_t* only_big, hipStream_t st);
// Exclusive scan of the per-grid totals into nei_off (u64, ncell + 1); total into the header.
hipError_t launch_nei_offsets(const GridView& g, const uint32_t* off_counts, uint64_t* nei_off, uint64_t* partial,
                              hipStream_t st);
// Pass 2: write Nei(g) (skipped, with kErrNeiOverflow, if the total exceeds
// `capacity` entries).  nei_up (ncell entries): for lists in walk order,
// the range [x, y) of Nei(g), relative to its start, that holds exactly the
// neighbours of larger index (the other orders leave it alone).
hipError_t launch_nei_fill(const GridView& g, const NeiQuery& nq, const uint32_t* off_counts, const uint32_t* lane_cnt,
                           const uint64_t* nei_off, uint32_t* nei, uint64_t capacity, const uint32_t* only_big,
                           uint2* nei_up, hipStream_t st);
// Identifier -> grid index table (2^bits + 1 slots of 8 or 16 bytes, as
// output_table_bytes) for the hashing query; skeys: sorted identifiers.
hipError_t launch_grid_table(const GridView& g, const void* skeys, int key_bytes, void* table, int bits,
                             hipStream_t st);

// ---- core.hip
// Core sets s_i as runs of point rows.  A grid whose points are all core
// (every dense grid, and most others) uses its own sorted rows; only a grid
// holding both core and non-core points gets its core rows copied, in
// sorted order, to the side area behind row n.
struct CoreOut {
    uint8_t* core;              // n, sorted order
    uint32_t* core_cnt;         // ncell: core points of each grid (m_i)
    uint32_t* core_begin;       // ncell: first row of each grid's core set
    int32_t* ccrd;              // the row space: rows [0, n) = GridView::crd, then the side area
    uint32_t* corig;            // row -> global input index (rows [0, n) = the sorted index)
    uint32_t* side_off;         // ncell + 1: exclusive scan of the side rows of each grid
    uint32_t* cell_min_core;    // ncell: smallest input index of a core point (kNone if none)
    uint32_t* counts;           // header counts
    uint32_t* count_part;       // 5 words per workgroup of core_cells_kernel (ncell / 256 + 1 workgroups)
};
constexpr uint32_t kTinyCore = 8;  // core sets decided by one lane in the merge step
// Work counters of core marking (one copy per stat slot).
struct CoreStats {
    unsigned long long dists;   // distances evaluated
    unsigned long long points;  // candidate points streamed (once per batch of 64 queries)
    unsigned long long grids;   // neighbour grids opened
};
// Core flags (sorted order) and m_i per grid.  max_eps: the largest eps in
// the batch (small ones allow packed 16-bit coordinate differences);
// min_minpts: the smallest MinPts in the batch (large ones take two
// candidate rows per lane per step).  prune (used at d <= 4): test large
// neighbour grids' cells against the open queries before streaming them,
// for data whose grids hold a thousand points and more.
hipError_t launch_core_mark(const GridView& g, const uint64_t* nei_off, const uint32_t* nei, uint8_t* core,
                            uint32_t* core_cnt, CoreStats* stats, int64_t max_eps, int64_t min_minpts, bool prune,
                            hipStream_t st);
// Whether core marking compares coordinates as packed 16-bit differences
// for a batch whose largest eps is max_eps (exact for eps <= 10000: points
// of neighbouring grids differ by less than 2.13 eps per coordinate).
constexpr int64_t kPackedEpsMax = 10000;
inline bool core_mark_packed(int64_t max_eps) { return max_eps <= kPackedEpsMax; }
hipError_t launch_core_compact(const GridView& g, const CoreOut& c, uint32_t* partial, hipStream_t st);
// LDF order (Section 5.2): core grids by ascending core count (ties by grid
// index); rank[g] = (position (kNone for non-core grids), core_begin,
// core_cnt, 0).  ncc: number of
// core grids, or an upper bound (then pad_tail: the slots past the device
// count sort last, under the key 2^count_bits - 1); count_bits: bits of the
// sort keys.  Also sets parent[g] = g (union-find roots) and root_min[g] =
// kNone for every grid (the labelling step's minima).
hipError_t launch_ldf_order(const GridView& g, const CoreOut& c, bool by_count, int64_t ncc, int count_bits,
                            bool pad_tail, uint32_t* list, uint4* rank, uint32_t* parent, uint32_t* root_min,
                            uint32_t* keys_a, uint32_t* keys_b, uint32_t* vals_b, uint32_t* radix_scratch,
                            uint32_t* partial, uint32_t** sorted_list, hipStream_t st);

// ---- merge.hip (Algorithms 4-5, union-find)
constexpr int kStatSlots = 64;  // copies of each device counter (see MergeStats)
struct MergeStats {
    unsigned long long pairs, skipped, tests, yes, iters, max_iters, dists, set_points;
};
// wide (here and below): the batch's largest eps exceeds GD_EPS_MAX, and
// squared distances are taken in 64 bits against Inst::T64 / Tm64.
// Largest core set the merge kernels' LDS bitmaps hold.  A pair with a
// larger set is queued (HugeQueue) and tested by merge_heavy_kernel, whose
// bitmaps live in device memory.
constexpr int64_t kMaxCoreBits = 262144;
// Core sets from this size on are merged by a workgroup of kCoopWaves waves
// per pair (in eager runs; graph replays keep one wave per grid).
constexpr int64_t kHeavyCore = 8192;
constexpr int kCoopWaves = 8;
// Pairs (g_i, g_j) deferred by the LDS kernels.  pairs == nullptr: no queue
// (a planned run); meeting a larger set then raises kErrCoreCap.
struct HugeQueue {
    uint2* pairs;
    uint32_t cap;
    uint32_t* count;  // appended so far (may pass cap: then kErrCoreCap is raised)
};
struct CellSummary;
// waves: waves per workgroup of the FastMerging kernel (1, 2 or 4; fewer
// if the LDS bitmaps do not fit).  small_lanes: lanes per grid of the
// tiny-set kernel (16: four grids per wave; else 64).  n_small: tiny core grids leading the
// visiting order (-2: as many as the device count says, -1: not ordered).
// tiny_done: the pairs of two tiny core sets were already merged (walk mode).
// nei_up (optional, lists in walk order): each list's range of larger-index
// neighbours (launch_nei_fill), the only ones the tiny-set kernel tests.
hipError_t launch_merge(const GridView& g, const CoreOut& c, const uint64_t* nei_off, const uint32_t* nei,
                        const uint2* nei_up,
                        const uint32_t* ldf_list, const uint4* rank, int64_t n_core_cells, int64_t n_small,
                        int64_t max_core, int waves, int small_lanes, bool tiny_done, const HugeQueue& huge,
                        bool wide,
                        uint32_t* parent, MergeStats* stats, const __half* proposal, const CellSummary* sum,
                        hipStream_t st);
// Sum over core grids with at least kHeavyCore core points of |Nei(g)| + 1
// (added to *sum; the caller clears it): with both orders no pair is queued
// twice from one side, so twice this bounds the queue.
hipError_t launch_huge_scan(const GridView& g, const CoreOut& c, const uint64_t* nei_off, unsigned long long* sum,
                            hipStream_t st);
// Tests the queued pairs (FastMerging, union on yes) with `blocks`
// workgroups of kCoopWaves waves, each with 2 * words words of device memory
// at slabs.  bfs: the pair's second grid is claimed for the search (state,
// next, cnt[2]) as in the BFS level kernel.
hipError_t launch_merge_huge(const GridView& g, const CoreOut& c, const HugeQueue& huge, uint64_t* slabs,
                             uint32_t words, uint32_t blocks, bool bfs, bool wide, uint32_t* state, uint32_t* next,
                             uint32_t* cnt, uint32_t* parent, MergeStats* stats, hipStream_t st);
// The BFS order of Algorithm 6 (GD_OPT_MERGE_ORDER = 2), on the full lists.
// state: ncell u32, cleared to 0 for every grid first.  cnt: 3 u32 (the
// caller clears them): cnt[0] unclassified core grids seen by the seed pass,
// cnt[1] seeds appended to front, cnt[2] grids appended to next by a level.
hipError_t launch_bfs_seeds(const GridView& g, const CoreOut& c, const uint64_t* nei_off, const uint32_t* nei,
                            uint32_t* state, uint32_t* front, uint32_t* cnt, hipStream_t st);
hipError_t launch_bfs_level(const GridView& g, const CoreOut& c, const uint64_t* nei_off, const uint32_t* nei,
                            const uint32_t* front, uint32_t nfront, uint32_t* next, uint32_t* cnt, int64_t max_core,
                            const HugeQueue& huge, bool wide, uint32_t* state, uint32_t* parent, MergeStats* stats,
                            hipStream_t st);
// pts: d x m SoA; rows: scratch of m rows (row_stride(d) int32 each).
hipError_t launch_merge_pairs(const int32_t* pts, int64_t m, int d, int32_t* rows, const uint32_t* pairs,
                              int64_t npairs, int64_t eps, uint32_t max_count, uint8_t* answers, uint32_t* iterations,
                              hipStream_t st);
// root_min must hold kNone for every grid (launch_ldf_order clears it).
hipError_t launch_labels(const GridView& g, const CoreOut& c, uint32_t* parent, uint32_t* root_min,
                         int32_t* cell_label, hipStream_t st);

// ---- learned.hip (the learned proposal)
hipError_t launch_summaries(const GridView& g, const CoreOut& c, CellSummary* out, hipStream_t st);
hipError_t launch_harvest(const GridView& g, const CoreOut& c, const CellSummary* sum, const uint64_t* nei_off,
                          const uint32_t* nei, uint32_t seed, uint32_t keep_mod, int64_t cap, int64_t max_core,
                          __half* X, float* Tg, float* C, unsigned long long* counter, hipStream_t st);
hipError_t launch_mlp_forward(const __half* X, int64_t B, const __half* params, float* Z, hipStream_t st);
struct TrainArgs;
hipError_t launch_mlp_train(const TrainArgs& a, hipStream_t st);

// ---- walk.hip (consumers that walk the grid tree themselves; no Nei lists)
// Core flags and m_i per grid, each sparse grid's queries counting hits over
// the neighbours its own tree walk finds, with early exit at MinPts.
hipError_t launch_core_walk(const GridView& g, const TreeView& t, uint8_t* core, uint32_t* core_cnt, CoreStats* stats,
                            bool wide, hipStream_t st);
// Pairs of tiny core sets (both at most kTinyCore points), each tested once
// from its lower grid; n_small as for launch_merge.  Pairs involving a larger
// core set are left to launch_merge (with lists for those grids only).
hipError_t launch_merge_walk(const GridView& g, const CoreOut& c, const TreeView& t, const uint32_t* ldf_list,
                             int64_t n_small, uint32_t* parent, MergeStats* stats, bool wide, hipStream_t st);
// Border and noise points of the grids holding a non-core point.
hipError_t launch_border_walk(const GridView& g, const CoreOut& c, const TreeView& t, const int32_t* cell_label,
                              bool wide, hipStream_t st);

// ---- border.hip
// Grids with a non-core point: border search and output through the permutation.
// lanes: 16 serves four grids per wave side by side; otherwise a wave per
// grid (a wave checks 64 grids when there are millions of them).
hipError_t launch_output(const GridView& g, const CoreOut& c, const uint64_t* nei_off, const uint32_t* nei,
                         const int32_t* cell_label, bool wide, int lanes, hipStream_t st);
// All-core grids: output in input order through an identifier -> label hash
// table of 2^bits slots (+1) in `table` (output_table_bytes).  keys_in: the
// identifiers in input order, shifted up by key_lo bits (the packed-row
// words of launch_keys_packed64; else 0); skeys: sorted.
template <typename K>
hipError_t launch_output_direct(const GridView& g, const CoreOut& c, const K* keys_in, const K* skeys,
                                const int32_t* cell_label, void* table, int bits, int key_lo, hipStream_t st);
size_t output_table_bytes(int bits, int key_bytes);
// All-core grids of identifiers wider than 64 bits: output through the
// sort permutation (no hash table).
hipError_t launch_output_allcore(const GridView& g, const CoreOut& c, const int32_t* cell_label, hipStream_t st);

}  // namespace gd
