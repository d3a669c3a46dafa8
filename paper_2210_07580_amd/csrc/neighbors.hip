// Non-empty neighbouring grids query (Section 4.2.2, Algorithm 3, Eq. (2)).
//
// Each grid g walks the grid tree level by level (after the exact match of
// g's instance at level 0), its first levels split over lanes.  At level l
// it visits the children whose key k satisfies |k - g_l| <= w, accumulating
//   offset += max(|k - g_l| - 1, 0)^2                       (Eq. (2))
// and drops a node once offset >= d.  The paper scans the fixed window
// +-ceil(sqrt(d)) and prunes afterwards; here the window shrinks with the
// budget left (w = 1 + isqrt(d - 1 - offset)), which keeps exactly the same
// nodes.  The first child in the window is found by binary search over the
// node's contiguous, ascending children (the role the paper gives to its
// hash table h for nodes with many children).  The result excludes g itself
// and is ordered by offset (the paper's counting sort), nearest grids first.
#include "launch.hpp"
#include "scan.hpp"

namespace gd {

// Levels 1..D of the walk (level 0, the instance, is matched exactly by the
// caller).  `g` holds the query grid's identifiers at g[1..D]; `dk` is the
// instance's own dimension (identifier rows beyond dk are 0 for all its grids).
template <int D, int L, typename Emit>
__device__ __forceinline__ void walk(const TreeView& t, const int32_t (&g)[D + 1], int dk, uint32_t lo, uint32_t hi,
                                     int off, Emit& emit) {
    const int R = dk - off;  // budget left, >= 1
    int gmax = 0;
    while ((gmax + 1) * (gmax + 1) <= R - 1) ++gmax;
    const int win = gmax + 1;
    const int32_t* __restrict__ key = t.key[L];
    const int32_t lo_key = g[L] - win;
    uint32_t a = lo, b = hi;
    while (a < b) {
        const uint32_t m = (a + b) >> 1;
        if (key[m] < lo_key) a = m + 1; else b = m;
    }
    for (; a < hi; ++a) {
        const int32_t dk_ = key[a] - g[L];
        if (dk_ > win) break;
        const int gap = (dk_ < 0 ? -dk_ : dk_) - 1;
        const int o = off + (gap > 0 ? gap * gap : 0);
        if (o >= dk) continue;
        if constexpr (L == D) {
            emit(a, o);
        } else {
            walk<D, L + 1>(t, g, dk, t.child[L][a], t.child[L][a + 1], o, emit);
        }
    }
}

// With few grids, each grid's walk is split over kSplit = 8 consecutive
// lanes: lane p takes the level-1 children whose key is g_1 + p - 3.  The
// level-1 window is 1 + isqrt(d - 1) <= 3 for d <= 8, so offsets -3..+3
// cover it (lane 7 has nothing to do).  The tree walk is a chain of
// dependent loads, and one thread per grid leaves most of the chip idle when
// the grids number in the tens of thousands; with millions of grids one
// thread per grid is already enough and the split would only add the extra
// counting walk of the fill pass.  (Splitting the next level too repeats the
// upper searches in every lane and costs more than it saves.)  Lanes follow
// the tree order, so the lists come out as one walk would emit them.
constexpr int kSplit = 8;
constexpr int64_t kSplitMaxGrids = 1 << 20;

inline int nei_lanes(int64_t ncell) { return ncell <= kSplitMaxGrids ? kSplit : 1; }

__device__ __forceinline__ int level_window(int budget) {
    int w = 0;
    while ((w + 1) * (w + 1) <= budget - 1) ++w;
    return w + 1;
}

// First index in [lo, hi) whose key is >= want.
__device__ __forceinline__ uint32_t lower_key(const int32_t* __restrict__ key, uint32_t lo, uint32_t hi, int32_t want) {
    while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if (key[m] < want) lo = m + 1; else hi = m;
    }
    return lo;
}

// The neighbours below the level-1 children with key g_1 + delta,
// delta in [d_lo, d_hi].
template <int D, typename Emit>
__device__ __forceinline__ void query_part(const TreeView& t, const int32_t (&g)[D + 1], int dk, int d_lo, int d_hi,
                                           Emit& emit) {
    const int w1 = level_window(dk);
    d_lo = d_lo < -w1 ? -w1 : d_lo;
    d_hi = d_hi > w1 ? w1 : d_hi;
    if (d_lo > d_hi) return;
    const uint32_t a0 = lower_key(t.key[0], 0, t.level_count[0], g[0]);
    const uint32_t hi1 = t.child[0][a0 + 1];
    const int32_t* __restrict__ key1 = t.key[1];
    for (uint32_t a = lower_key(key1, t.child[0][a0], hi1, g[1] + d_lo); a < hi1; ++a) {
        const int d1 = key1[a] - g[1];
        if (d1 > d_hi) break;
        const int gap = (d1 < 0 ? -d1 : d1) - 1;
        const int o = gap > 0 ? gap * gap : 0;
        if (o >= dk) continue;
        if constexpr (D == 1) {
            emit(a, o);
        } else {
            walk<D, 2>(t, g, dk, t.child[1][a], t.child[1][a + 1], o, emit);
        }
    }
}

template <int D>
__device__ __forceinline__ void load_grid(const GridView& gv, int64_t c, int32_t (&g)[D + 1]) {
#pragma unroll
    for (int j = 0; j <= D; ++j) g[j] = gv.ck[(int64_t)j * gv.ck_stride + c];
}

// This lane's part of grid c's neighbours, counted per offset value into
// cnt[o][threadIdx.x] (LDS).
template <int D, int P>
__device__ __forceinline__ void count_part(const GridView& gv, const TreeView& t, int64_t c, int p,
                                           uint32_t (*cnt)[kBlock]) {
    int32_t g[D + 1];
    load_grid<D>(gv, c, g);
    const int dk = gv.b.inst[g[0]].d;
    auto emit = [&](uint32_t a, int o) {
        if (a != (uint32_t)c) cnt[o][threadIdx.x] += 1;
    };
    query_part<D>(t, g, dk, P == 1 ? -3 : p - 3, P == 1 ? 3 : p - 3, emit);
}

// With lane_cnt (split walks only), each lane also keeps its own counts for
// the fill pass, which then needs no second counting walk.
template <int D, int P>
__global__ __launch_bounds__(kBlock) void nei_count_kernel(GridView gv, TreeView t, uint32_t* __restrict__ off_counts,
                                                           uint32_t* __restrict__ lane_cnt) {
    __shared__ uint32_t sc[D][kBlock];
    const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t c = gt / P;
    const int p = (int)(gt % P);
    const bool valid = c < (int64_t)*gv.ncell_dev;
    if (P == 1 && !valid) return;
#pragma unroll
    for (int o = 0; o < D; ++o) sc[o][threadIdx.x] = 0;
    if (valid) count_part<D, P>(gv, t, c, p, sc);
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

// The list of grid c holds its offset-0 neighbours, then offset 1, ...; within
// one offset value the lanes' parts follow each other in lane order.  With a
// split, each lane first counts its part again to find where its entries go.
// With one lane per grid (long lists per lane), found neighbours are staged
// in LDS and stored kFillStage at a time: gfx9 counts outstanding vector
// loads and stores with one in-order counter, so a store issued between two
// loads of the tree walk would make the second wait for it; in bursts, the
// walk waits once per kFillStage entries (cfg2-like data: 59 -> 52 ms; 4
// entries gave 56 ms, 16 cost occupancy and gave 68 ms).  A split walk
// emits a few entries per lane, and staging them only costs.
constexpr int kFillStage = 8;

template <int D, int P>
__global__ __launch_bounds__(kBlock) void nei_fill_kernel(GridView gv, TreeView t, const uint32_t* __restrict__ off_counts,
                                                          const uint32_t* __restrict__ lane_cnt,
                                                          const uint64_t* __restrict__ nei_off, uint32_t* __restrict__ nei,
                                                          uint64_t capacity) {
    __shared__ uint32_t pos[D][kBlock];
    constexpr int kStage = P == 1 ? kFillStage : 1;
    __shared__ uint32_t stage_a[kStage][kBlock];
    __shared__ uint8_t stage_o[kStage][kBlock];
    const int64_t ncell = *gv.ncell_dev;
    if (nei_off[ncell] > capacity) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&gv.b.hdr->err, kErrNeiOverflow);
        return;
    }
    const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t c = gt / P;
    const int p = (int)(gt % P);
    const bool valid = c < ncell;
    if (P == 1 && !valid) return;
    if constexpr (P > 1) {
        if (lane_cnt) {
#pragma unroll
            for (int o = 0; o < D; ++o) pos[o][threadIdx.x] = valid ? lane_cnt[gt * D + o] : 0u;
        } else {
#pragma unroll
            for (int o = 0; o < D; ++o) pos[o][threadIdx.x] = 0;
            if (valid) count_part<D, P>(gv, t, c, p, pos);
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
    load_grid<D>(gv, c, g);
    const int dk = gv.b.inst[g[0]].d;
    int staged = 0;
    auto flush = [&]() {
        for (int j = 0; j < staged; ++j) {
            const uint32_t a = stage_a[j][threadIdx.x];
            const int o = stage_o[j][threadIdx.x];
            const uint32_t k = pos[o][threadIdx.x];
            pos[o][threadIdx.x] = k + 1;
            nei[base + k] = a;
        }
        staged = 0;
    };
    auto emit = [&](uint32_t a, int o) {
        if (a == (uint32_t)c) return;
        if constexpr (P == 1) {
            stage_a[staged][threadIdx.x] = a;
            stage_o[staged][threadIdx.x] = (uint8_t)o;
            if (++staged == kStage) flush();
        } else {
            const uint32_t k = pos[o][threadIdx.x];
            pos[o][threadIdx.x] = k + 1;
            nei[base + k] = a;
        }
    };
    query_part<D>(t, g, dk, P == 1 ? -3 : p - 3, P == 1 ? 3 : p - 3, emit);
    flush();
}

int64_t nei_lane_count_words(int64_t ncell, int D) {
    return nei_lanes(ncell) > 1 ? ncell * kSplit * D : 0;
}

hipError_t launch_nei_count(const GridView& g, const TreeView& t, uint32_t* off_counts, uint32_t* lane_cnt,
                            hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    if (nei_lanes(g.ncell) > 1) {
        GD_DISPATCH_D(g.D, (nei_count_kernel<D, kSplit><<<dim3(grid_for(g.ncell * kSplit)), dim3(kBlock), 0, st>>>(
                               g, t, off_counts, lane_cnt)));
    } else {
        GD_DISPATCH_D(g.D, (nei_count_kernel<D, 1><<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(
                               g, t, off_counts, nullptr)));
    }
    return hipGetLastError();
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

hipError_t launch_nei_fill(const GridView& g, const TreeView& t, const uint32_t* off_counts, const uint32_t* lane_cnt,
                           const uint64_t* nei_off, uint32_t* nei, uint64_t capacity, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    if (nei_lanes(g.ncell) > 1) {
        GD_DISPATCH_D(g.D, (nei_fill_kernel<D, kSplit><<<dim3(grid_for(g.ncell * kSplit)), dim3(kBlock), 0, st>>>(
                               g, t, off_counts, lane_cnt, nei_off, nei, capacity)));
    } else {
        GD_DISPATCH_D(g.D, (nei_fill_kernel<D, 1><<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(
                               g, t, off_counts, nullptr, nei_off, nei, capacity)));
    }
    return hipGetLastError();
}

}  // namespace gd
