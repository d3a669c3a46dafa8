// Host-side launchers of the pipeline phases, shared between the
// translation units.  Every launcher takes plain device pointers and a
// stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gd {

constexpr int kMaxD = 8;

// Error bits raised by kernels into the device error word.
enum : uint32_t {
    kErrNotInteger = 1u,   // a coordinate is not a finite integer of magnitude <= 2^24
};

struct KeyParams {
    int d;
    int64_t eps;
    int mn[kMaxD];     // per-dimension minimum of the input
    int bits[kMaxD];   // bits of the identifier in each dimension
    int shift[kMaxD];  // position of dimension j's field (dimension 0 highest)
};

// Grid tree (Section 4.2.1) as flat level arrays.  Level l (0-based, l < d)
// holds one node per distinct identifier prefix of length l+1, in
// lexicographic order; key[l][a] is the node's identifier in dimension l.
// For l < d-1 the children of node a are the level-(l+1) nodes
// [child[l][a], child[l][a+1]); level d-1 nodes are the grids themselves.
struct TreeView {
    const int32_t* key[kMaxD];
    const uint32_t* child[kMaxD];
    const uint32_t* level_count;  // device: nodes per level (level 0 = root's children)
};

// Sorted points and grids.
struct GridView {
    int64_t n;
    int d;
    int64_t T;                 // eps^2
    int minpts;
    const int32_t* crd;        // d x n, SoA: coordinate minus the minimum, sorted by grid
    const uint32_t* sidx;      // n: input index of each sorted point
    int64_t ncell;
    const uint32_t* cell_start;  // ncell + 1
    const int32_t* ck;         // d x ck_stride: grid identifiers, SoA
    int64_t ck_stride;
};

// ---- partition.hip
hipError_t launch_minmax(const float* x, int64_t n, int d, int* mn, int* mx, uint32_t* err, hipStream_t st);
template <typename K>
hipError_t launch_keys(const float* x, int64_t n, const KeyParams& kp, K* keys, hipStream_t st);
hipError_t launch_gather(const float* x, int64_t n, const KeyParams& kp, const uint32_t* sidx, int32_t* crd,
                         hipStream_t st);
// Runs of equal keys: cell_start[0..ncell], cell_of[n]; *ncell_dev written.
template <typename K>
hipError_t launch_cells(const K* skeys, int64_t n, const KeyParams& kp, uint32_t* excl, uint32_t* partial,
                        uint32_t* ncell_dev, uint32_t* cell_start, uint32_t* cell_of, int32_t* ck, int64_t ck_stride,
                        hipStream_t st);
// Grid tree levels over the ncell sorted grids.  level_excl: d x (ncell+1)
// scratch; keys / child arrays are written into the given level buffers.
hipError_t launch_tree(const GridView& g, const KeyParams& kp, uint32_t* level_excl, uint32_t* partial,
                       uint32_t* level_count_dev, int32_t* const* tkey, uint32_t* const* tchild, hipStream_t st);

// ---- neighbors.hip (Algorithm 3)
// Pass 1: per-grid neighbour count per offset value (ncell x d, u32) and in total.
hipError_t launch_nei_count(const GridView& g, const TreeView& t, uint32_t* off_counts, hipStream_t st);
// Exclusive scan of the per-grid totals into nei_off (u64, ncell + 1).
hipError_t launch_nei_offsets(const GridView& g, const uint32_t* off_counts, uint64_t* nei_off, uint64_t* partial,
                              hipStream_t st);
// Pass 2: write Nei(g) ordered by offset.
hipError_t launch_nei_fill(const GridView& g, const TreeView& t, const uint32_t* off_counts, const uint64_t* nei_off,
                           uint32_t* nei, hipStream_t st);

// ---- core.hip
struct CoreOut {
    uint8_t* core;              // n, sorted order
    uint32_t* core_excl;        // n + 1: exclusive scan of core flags
    uint32_t* core_start;       // ncell + 1: first compacted core point of each grid
    int32_t* ccrd;              // core points' coordinates, compacted, cstride int32 per point
    int cstride;                // 4 (d <= 4) or 8: padded point record
    uint32_t* corig;            // n: input index of each compacted core point
    uint32_t* cell_min_core;    // ncell: smallest input index of a core point (kNone if none)
    uint32_t* counts;           // device counters: [0] ncore, [1] ncorecell, [2] max core/grid, [3] dense grids,
                                // [4] core grids with at most kTinyCore core points
};
hipError_t launch_core_mark(const GridView& g, const uint64_t* nei_off, const uint32_t* nei, uint8_t* core,
                            unsigned long long* dist_counter, hipStream_t st);
hipError_t launch_core_compact(const GridView& g, const CoreOut& c, uint32_t* partial, hipStream_t st);
// LDF order (Section 5.2): core grids by ascending core count (ties by grid
// index); rank[g] = position (kNone for non-core grids).  Needs ncell-sized
// scratch buffers.
hipError_t launch_ldf_order(const GridView& g, const CoreOut& c, bool by_count, int64_t ncc, int count_bits,
                            uint32_t* list, uint32_t* rank, uint32_t* keys_a, uint32_t* keys_b, uint32_t* vals_b,
                            uint32_t* radix_scratch, uint32_t* excl, uint32_t* partial, uint32_t** sorted_list,
                            hipStream_t st);

// ---- merge.hip (Algorithms 4-5, union-find)
constexpr int kStatSlots = 64;  // copies of each device counter (see MergeStats)
struct MergeStats {
    unsigned long long pairs, skipped, tests, yes, iters, max_iters, dists, set_points;
};
enum : uint32_t {
    kErrMergeRunaway = 2u,  // FastMerging exceeded its iteration bound (cannot happen; checked anyway)
};
// Largest core set a grid may hold (LDS bitmaps of the merge step).
constexpr int64_t kMaxCoreBits = 262144;
constexpr uint32_t kTinyCore = 8;  // core sets decided by one lane in the merge step
hipError_t launch_merge(const GridView& g, const CoreOut& c, const uint64_t* nei_off, const uint32_t* nei,
                        const uint32_t* ldf_list, const uint32_t* rank, int64_t n_core_cells, int64_t n_small,
                        int64_t max_core, int64_t eps, uint32_t* parent, MergeStats* stats, uint32_t* err,
                        hipStream_t st);
hipError_t launch_merge_pairs(const int32_t* pts, int64_t m, int d, const uint32_t* pairs, int64_t npairs,
                              int64_t eps, uint32_t max_count, uint8_t* answers, uint32_t* iterations,
                              hipStream_t st);
hipError_t launch_labels(const GridView& g, const CoreOut& c, uint32_t* parent, uint32_t* root_min,
                         int32_t* cell_label, hipStream_t st);

// ---- border.hip
hipError_t launch_output(const GridView& g, const CoreOut& c, const uint64_t* nei_off, const uint32_t* nei,
                         const int32_t* cell_label, int32_t* labels, uint8_t* core_flags, hipStream_t st);

}  // namespace gd
