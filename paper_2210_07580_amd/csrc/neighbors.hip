// Non-empty neighbouring grids query (Section 4.2.2, Algorithm 3, Eq. (2)),
// written out as lists Nei(g).
//
// Two queries produce the same sets:
//   the grid tree (Algorithm 3): each grid walks the tree level by level
//     (walk.hpp), its first level split over lanes;
//   direct hashing, for comparison: every candidate identifier g' with
//     sum_j max(|g'_j - g_j| - 1, 0)^2 < d (the same shrinking windows,
//     enumerated over all integers rather than over existing tree nodes) is
//     probed in a hash table of the non-empty grids.
// The result excludes g itself.  It is ordered by offset (the paper's
// counting sort, nearest grids first, for early exit in core marking) when
// the query splits over lanes or hashes; a one-lane tree walk over millions
// of grids, or on request, keeps walk order: level-1 keys g_1, g_1 + 1, ..,
// g_1 + 3, then g_1 - 1, .., g_1 - 3, each subtree in ascending order, so
// that the neighbours with a larger index form one range per list (kept in
// nei_up for the merge of tiny core sets, which tests only those).
#include <algorithm>
#include <type_traits>

#include "hash.hpp"
#include "launch.hpp"
#include "scan.hpp"
#include "walk.hpp"

namespace gd {

// With few grids, each grid's query is split over kSplit = 8 consecutive
// lanes: lane p takes the level-1 key g_1 + p - 3.  The level-1 window is
// 1 + isqrt(d - 1) <= 3 for d <= 8, so offsets -3..+3 cover it (lane 7 has
// nothing to do).  The tree walk is a chain of dependent loads, and one
// thread per grid leaves most of the chip idle when the grids number in the
// tens of thousands; with millions of grids one thread per grid is already
// enough and the split would only add the extra counting walk of the fill
// pass.  (Splitting the next level too repeats the upper searches in every
// lane and costs more than it saves.)  Lanes follow the query order, so the
// lists come out as one query would emit them.
constexpr int kSplit = 8;
constexpr int64_t kSplitMaxGrids = 1 << 20;

inline int nei_lanes(int64_t ncell) { return ncell <= kSplitMaxGrids ? kSplit : 1; }

// Algorithm 3 on the grid tree.
struct TreeQuery {
    TreeView t;
    // The neighbours below the level-1 children with key g_1 + delta, delta
    // in [d_lo, d_hi], in tree order (emit(a, offset) for each; g itself is
    // emitted too and the callers skip it).
    template <int D, typename Emit>
    __device__ __forceinline__ void part(const int32_t (&g)[D + 1], int dk, int d_lo, int d_hi, Emit& emit) const {
        const int w1 = walk_window(dk);
        d_lo = d_lo < -w1 ? -w1 : d_lo;
        d_hi = d_hi > w1 ? w1 : d_hi;
        if (d_lo > d_hi) return;
        auto visit = [&](uint32_t a, int o) -> bool {
            emit(a, o);
            return true;
        };
        const uint32_t a0 = walk_lower(t.key[0], 0, t.level_count[0], g[0]);
        const uint32_t hi1 = t.child[0][a0 + 1];
        const int32_t* __restrict__ key1 = t.key[1];
        for (uint32_t a = walk_lower(key1, t.child[0][a0], hi1, g[1] + d_lo); a < hi1; ++a) {
            const int d1 = key1[a] - g[1];
            if (d1 > d_hi) break;
            const int gap = (d1 < 0 ? -d1 : d1) - 1;
            const int o = gap > 0 ? gap * gap : 0;
            if (o >= dk) continue;
            if constexpr (D == 1) {
                emit(a, o);
            } else {
                walk_levels<D, 2>(t, g, dk, t.child[1][a], t.child[1][a + 1], o, true, visit);
            }
        }
    }
};

// Direct hashing of every candidate identifier.  Identifiers are packed as
// in the identifier pass: the instance above inst_shift, coordinate j of
// the grid at shift[j] with bits[j] bits.
template <typename K>
struct HashQuery {
    const HashSlot<K>* tab;
    int bits;              // table of 2^bits slots (+1)
    const Inst* inst;      // device instance table
    const int* inst_shift; // device: position of the instance field

    template <int D, int L, typename Emit>
    __device__ __forceinline__ void probe(const Inst& I, const int32_t (&g)[D + 1], int dk, K key, int off,
                                          Emit& emit) const {
        const int win = walk_window(dk - off);
        const int64_t hi = (int64_t)1 << I.bits[L - 1];
        for (int32_t k = g[L] - win; k <= g[L] + win; ++k) {
            if (k < 0 || k >= hi) continue;
            const int dl = k - g[L];
            const int gap = (dl < 0 ? -dl : dl) - 1;
            const int o = off + (gap > 0 ? gap * gap : 0);
            if (o >= dk) continue;
            const K kk = key | ((K)(uint32_t)k << I.shift[L - 1]);
            if constexpr (L == D) {
                const int32_t a = grid_table_find<K>(tab, bits, kk);
                if (a >= 0) emit((uint32_t)a, o);
            } else {
                probe<D, L + 1>(I, g, dk, kk, o, emit);
            }
        }
    }

    template <int D, typename Emit>
    __device__ __forceinline__ void part(const int32_t (&g)[D + 1], int dk, int d_lo, int d_hi, Emit& emit) const {
        const Inst& I = inst[g[0]];
        const int ishift = *inst_shift;
        const K top = ishift >= (int)(8 * sizeof(K)) ? K(0) : (K)(uint32_t)g[0] << ishift;
        const int w1 = walk_window(dk);
        d_lo = d_lo < -w1 ? -w1 : d_lo;
        d_hi = d_hi > w1 ? w1 : d_hi;
        const int64_t hi = (int64_t)1 << I.bits[0];
        for (int d1 = d_lo; d1 <= d_hi; ++d1) {
            const int32_t k = g[1] + d1;
            if (k < 0 || k >= hi) continue;
            const int gap = (d1 < 0 ? -d1 : d1) - 1;
            const int o = gap > 0 ? gap * gap : 0;
            if (o >= dk) continue;
            const K kk = top | ((K)(uint32_t)k << I.shift[0]);
            if constexpr (D == 1) {
                const int32_t a = grid_table_find<K>(tab, bits, kk);
                if (a >= 0) emit((uint32_t)a, o);
            } else {
                probe<D, 2>(I, g, dk, kk, o, emit);
            }
        }
    }
};

// This lane's part of grid c's neighbours, counted per offset value into
// cnt[o][threadIdx.x] (LDS).
template <int D, int P, typename Q>
__device__ __forceinline__ void count_part(const GridView& gv, const Q& q, int64_t c, int p, uint32_t (*cnt)[kBlock]) {
    int32_t g[D + 1];
    load_grid_key<D>(gv, c, g);
    const int dk = gv.b.inst[g[0]].d;
    auto emit = [&](uint32_t a, int o) {
        if (a != (uint32_t)c) cnt[o][threadIdx.x] += 1;
    };
    q.template part<D>(g, dk, P == 1 ? -3 : p - 3, P == 1 ? 3 : p - 3, emit);
}

// only_big (optional): the core counts of the grids; then only grids with
// more than kTinyCore core points get a list (the others count 0).
__device__ __forceinline__ bool wants_list(const uint32_t* only_big, int64_t c) {
    return !only_big || only_big[c] > kTinyCore;
}

// With lane_cnt (split queries only), each lane also keeps its own counts
// for the fill pass, which then needs no second counting query.  kTotal
// (lists in walk order, one lane per grid): only the list length is needed,
// kept in a register and stored as the offset-0 count (the others 0).
template <int D, int P, bool kTotal, typename Q>
__global__ __launch_bounds__(kBlock) void nei_count_kernel(GridView gv, Q q, uint32_t* __restrict__ off_counts,
                                                           uint32_t* __restrict__ lane_cnt,
                                                           const uint32_t* __restrict__ only_big) {
    static_assert(!kTotal || P == 1, "totals are counted by one lane per grid");
    __shared__ uint32_t sc[kTotal ? 1 : D][kBlock];
    const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t c = gt / P;
    const int p = (int)(gt % P);
    const bool valid = c < (int64_t)*gv.ncell_dev;
    if (P == 1 && !valid) return;
    if constexpr (kTotal) {
        uint32_t total = 0;
        if (wants_list(only_big, c)) {
            int32_t g[D + 1];
            load_grid_key<D>(gv, c, g);
            const int dk = gv.b.inst[g[0]].d;
            auto emit = [&](uint32_t a, int) { total += a != (uint32_t)c ? 1u : 0u; };
            q.template part<D>(g, dk, -3, 3, emit);
        }
#pragma unroll
        for (int o = 0; o < D; ++o) off_counts[c * D + o] = o == 0 ? total : 0u;
        return;
    }
#pragma unroll
    for (int o = 0; o < D; ++o) sc[o][threadIdx.x] = 0;
    if (valid && wants_list(only_big, c)) count_part<D, P>(gv, q, c, p, sc);
#pragma unroll
    for (int o = 0; o < D; ++o) {
        uint32_t v = sc[o][threadIdx.x];
        if (P > 1 && lane_cnt && valid) lane_cnt[gt * D + o] = v;
        // sum over the grid's lanes (every lane takes part in the shuffles)
#pragma unroll
        for (int s = 1; s < P; s <<= 1) v += __shfl_xor(v, s);
        if (valid && p == 0) off_counts[c * D + o] = v;
    }
}

// Ordered lists hold a grid's offset-0 neighbours, then offset 1, ...; within
// one offset value the lanes' parts follow each other in lane order.  In
// walk order (one lane per grid), found neighbours are staged in LDS and
// stored kFillStage consecutive entries at a time, so that the stores fill
// whole cache lines rather than scattering single words over offset buckets
// (with millions of grids the stores dominated this pass).  These runs are
// stored non-temporally: lists of millions of grids outgrow the caches, and
// streaming them past L2 keeps the grid tree, which the walks re-read, in
// cache (cfg2: 36 -> 33 ms).  The ordered lists' scattered single words are
// not, since they need L2 to gather them into lines (H: 3x slower).
// (Staging 32 entries and storing whole aligned lines with 16-byte stores
// was slower: more LDS and registers per lane cost the walk occupancy.)
constexpr int kFillStage = 16;

template <int D, int P, bool kOrdered, typename Q>
__global__ __launch_bounds__(kBlock) void nei_fill_kernel(GridView gv, Q q, const uint32_t* __restrict__ off_counts,
                                                          const uint32_t* __restrict__ lane_cnt,
                                                          const uint64_t* __restrict__ nei_off, uint32_t* __restrict__ nei,
                                                          uint64_t capacity, const uint32_t* __restrict__ only_big,
                                                          uint2* __restrict__ nei_up) {
    static_assert(kOrdered || P == 1, "walk order is written by one lane per grid");
    __shared__ uint32_t pos[D][kBlock];
    constexpr int kStage = kOrdered ? 1 : kFillStage;
    __shared__ uint32_t stage_a[kStage][kBlock];
    const int64_t ncell = *gv.ncell_dev;
    if (nei_off[ncell] > capacity) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&gv.b.hdr->err, kErrNeiOverflow);
        return;
    }
    const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t c = gt / P;
    const int p = (int)(gt % P);
    const bool valid = c < ncell && wants_list(only_big, c);
    if (P == 1 && !valid) return;
    if constexpr (P > 1) {
        if (lane_cnt) {
#pragma unroll
            for (int o = 0; o < D; ++o) pos[o][threadIdx.x] = valid ? lane_cnt[gt * D + o] : 0u;
        } else {
#pragma unroll
            for (int o = 0; o < D; ++o) pos[o][threadIdx.x] = 0;
            if (valid) count_part<D, P>(gv, q, c, p, pos);
        }
    }
    uint32_t run = 0;
#pragma unroll
    for (int o = 0; o < D; ++o) {
        uint32_t mine = 0, incl = 0;
        if constexpr (P > 1) {
            // inclusive sum over the grid's lanes up to this one
            mine = pos[o][threadIdx.x];
            incl = mine;
#pragma unroll
            for (int s = 1; s < P; s <<= 1) {
                const uint32_t v = __shfl_up(incl, s, P);
                if (p >= s) incl += v;
            }
        }
        pos[o][threadIdx.x] = run + (incl - mine);
        run += valid ? off_counts[c * D + o] : 0u;
    }
    if (!valid) return;
    const uint64_t base = nei_off[c];
    int32_t g[D + 1];
    load_grid_key<D>(gv, c, g);
    const int dk = gv.b.inst[g[0]].d;
    if constexpr (kOrdered) {
        auto emit = [&](uint32_t a, int o) {
            if (a == (uint32_t)c) return;
            const uint32_t k = pos[o][threadIdx.x];
            pos[o][threadIdx.x] = k + 1;
            nei[base + k] = a;
        };
        q.template part<D>(g, dk, P == 1 ? -3 : p - 3, P == 1 ? 3 : p - 3, emit);
    } else {
        uint32_t run_pos = 0;
        int staged = 0;
        auto flush = [&]() {
            for (int j = 0; j < staged; ++j)
                __builtin_nontemporal_store(stage_a[j][threadIdx.x], &nei[base + run_pos + j]);
            run_pos += (uint32_t)staged;
            staged = 0;
        };
        // level-1 keys g_1, g_1 + 1, .., g_1 + 3, then g_1 - 1, .., g_1 - 3,
        // each subtree ascending: the neighbours above g (larger identifier,
        // larger index) are the entries after g's own place in the first
        // run up to the start of the negative keys, one range [up_lo, up_hi)
        uint32_t up_lo = 0;
        auto emit = [&](uint32_t a, int) {
            if (a == (uint32_t)c) {
                up_lo = run_pos + (uint32_t)staged;
                return;
            }
            stage_a[staged][threadIdx.x] = a;
            if (++staged == kStage) flush();
        };
        q.template part<D>(g, dk, 0, 3, emit);
        const uint32_t up_hi = run_pos + (uint32_t)staged;
        for (int dlt = -1; dlt >= -3; --dlt) q.template part<D>(g, dk, dlt, dlt, emit);
        flush();
        nei_up[c] = make_uint2(up_lo, up_hi);
    }
}

// How the lists are produced (see the top of this file).
struct NeiShape {
    int P;         // lanes per grid
    bool ordered;  // by offset
};
inline NeiShape nei_shape(const NeiQuery& nq, int64_t ncell) {
    if (nq.kind == kNeiTreeWalkOrder) return {1, false};
    const int P = nei_lanes(ncell);
    return {P, nq.kind == kNeiHash || P > 1};
}

bool nei_walk_order(const NeiQuery& nq, int64_t ncell) { return !nei_shape(nq, ncell).ordered; }

int64_t nei_lane_count_words(const NeiQuery& nq, int64_t ncell, int D) {
    return nei_shape(nq, ncell).P > 1 ? ncell * kSplit * D : 0;
}

// Dispatch on the query (tree, or hash of 32- or 64-bit identifiers).
template <typename F>
hipError_t with_query(const NeiQuery& nq, F&& f) {
    if (nq.kind != kNeiHash) return f(TreeQuery{nq.t});
    if (nq.key_bytes == 4)
        return f(HashQuery<uint32_t>{reinterpret_cast<const HashSlot<uint32_t>*>(nq.table), nq.bits, nq.inst,
                                     nq.inst_shift});
    return f(HashQuery<uint64_t>{reinterpret_cast<const HashSlot<uint64_t>*>(nq.table), nq.bits, nq.inst,
                                 nq.inst_shift});
}

hipError_t launch_nei_count(const GridView& g, const NeiQuery& nq, uint32_t* off_counts, uint32_t* lane_cnt,
                            const uint32_t* only_big, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    const NeiShape sh = nei_shape(nq, g.ncell);
    return with_query(nq, [&](auto q) -> hipError_t {
        using Q = decltype(q);
        if (sh.P > 1) {
            GD_DISPATCH_D(g.D, (nei_count_kernel<D, kSplit, false, Q><<<dim3(grid_for(g.ncell * kSplit)),
                                                                        dim3(kBlock), 0, st>>>(g, q, off_counts,
                                                                                               lane_cnt, only_big)));
        } else if (!sh.ordered) {
            GD_DISPATCH_D(g.D, (nei_count_kernel<D, 1, true, Q><<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(
                                   g, q, off_counts, nullptr, only_big)));
        } else {
            GD_DISPATCH_D(g.D, (nei_count_kernel<D, 1, false, Q><<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(
                                   g, q, off_counts, nullptr, only_big)));
        }
        return hipGetLastError();
    });
}

struct CellTotal {
    const uint32_t* oc;
    const uint32_t* ncell;
    int D;
    __device__ uint64_t operator()(int64_t c) const {
        if (c >= (int64_t)*ncell) return 0;
        uint64_t s = 0;
        for (int o = 0; o < D; ++o) s += oc[c * D + o];
        return s;
    }
};

// nei_off[c] = ex; at c = ncell that is the total, kept in the header.
struct NeiOffWriter {
    uint64_t* nei_off;
    const uint32_t* ncell;
    uint64_t* total;
    __device__ void operator()(int64_t c, uint64_t ex, uint64_t) const {
        nei_off[c] = ex;
        if (c == (int64_t)*ncell) *total = ex;
    }
};

hipError_t launch_nei_offsets(const GridView& g, const uint32_t* off_counts, uint64_t* nei_off, uint64_t* partial,
                              hipStream_t st) {
    // nei_off[c] for c in [0, ncell]; entries beyond the true ncell repeat the total
    return scan_apply<uint64_t>(CellTotal{off_counts, g.ncell_dev, g.D}, g.ncell + 1,
                                NeiOffWriter{nei_off, g.ncell_dev, &g.b.hdr->nei_total}, (uint64_t*)nullptr, partial,
                                st);
}

hipError_t launch_nei_fill(const GridView& g, const NeiQuery& nq, const uint32_t* off_counts, const uint32_t* lane_cnt,
                           const uint64_t* nei_off, uint32_t* nei, uint64_t capacity, const uint32_t* only_big,
                           uint2* nei_up, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    const NeiShape sh = nei_shape(nq, g.ncell);
    return with_query(nq, [&](auto q) -> hipError_t {
        using Q = decltype(q);
        if (sh.P > 1) {
            GD_DISPATCH_D(g.D, (nei_fill_kernel<D, kSplit, true, Q><<<dim3(grid_for(g.ncell * kSplit)), dim3(kBlock),
                                                                      0, st>>>(g, q, off_counts, lane_cnt, nei_off, nei,
                                                                               capacity, only_big, nei_up)));
        } else if (sh.ordered) {
            GD_DISPATCH_D(g.D, (nei_fill_kernel<D, 1, true, Q><<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(
                                   g, q, off_counts, nullptr, nei_off, nei, capacity, only_big, nei_up)));
        } else if constexpr (std::is_same<Q, TreeQuery>::value) {
            GD_DISPATCH_D(g.D, (nei_fill_kernel<D, 1, false, Q><<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(
                                   g, q, off_counts, nullptr, nei_off, nei, capacity, only_big, nei_up)));
        } else {
            return hipErrorInvalidValue;  // hashing always writes ordered lists
        }
        return hipGetLastError();
    });
}

// The grid table of the hashing query: identifier -> grid index.
template <typename K>
__global__ __launch_bounds__(kBlock) void grid_table_build_kernel(const uint32_t* ncell, const uint32_t* cell_start,
                                                                  const K* __restrict__ skeys, HashSlot<K>* tab,
                                                                  int bits) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= (int64_t)*ncell) return;
    grid_table_insert<K>(tab, bits, skeys[cell_start[c]], (int32_t)c);
}

hipError_t launch_grid_table(const GridView& g, const void* skeys, int key_bytes, void* table, int bits,
                             hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    const int64_t slots = ((int64_t)1 << bits) + 1;
    const unsigned cb = (unsigned)std::min<int64_t>(grid_for(slots), 4096);
    if (key_bytes == 4) {
        auto* tab = reinterpret_cast<HashSlot<uint32_t>*>(table);
        hash_clear_kernel<uint32_t><<<dim3(cb), dim3(kBlock), 0, st>>>(tab, slots, -1);
        grid_table_build_kernel<uint32_t><<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(
            g.ncell_dev, g.cell_start, reinterpret_cast<const uint32_t*>(skeys), tab, bits);
    } else {
        auto* tab = reinterpret_cast<HashSlot<uint64_t>*>(table);
        hash_clear_kernel<uint64_t><<<dim3(cb), dim3(kBlock), 0, st>>>(tab, slots, -1);
        grid_table_build_kernel<uint64_t><<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(
            g.ncell_dev, g.cell_start, reinterpret_cast<const uint64_t*>(skeys), tab, bits);
    }
    return hipGetLastError();
}

}  // namespace gd
