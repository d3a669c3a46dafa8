// Non-empty neighbouring grids query (Section 4.2.2, Algorithm 3, Eq. (2)).
//
// One thread per grid g walks the grid tree level by level (after the
// exact match of g's instance at level 0).  At level l it
// visits the children whose key k satisfies |k - g_l| <= w, accumulating
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

// Full query: find the instance node at level 0, then walk levels 1..D.
template <int D, typename Emit>
__device__ __forceinline__ void query(const TreeView& t, const int32_t (&g)[D + 1], int dk, Emit& emit) {
    const int32_t* key0 = t.key[0];
    uint32_t a = 0, b = t.level_count[0];
    while (a < b) {
        const uint32_t m = (a + b) >> 1;
        if (key0[m] < g[0]) a = m + 1; else b = m;
    }
    walk<D, 1>(t, g, dk, t.child[0][a], t.child[0][a + 1], 0, emit);
}

template <int D>
__device__ __forceinline__ void load_grid(const GridView& gv, int64_t c, int32_t (&g)[D + 1]) {
#pragma unroll
    for (int j = 0; j <= D; ++j) g[j] = gv.ck[(int64_t)j * gv.ck_stride + c];
}

template <int D>
__global__ __launch_bounds__(kBlock) void nei_count_kernel(GridView gv, TreeView t, uint32_t* __restrict__ off_counts) {
    __shared__ uint32_t sc[D][kBlock];
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= (int64_t)*gv.ncell_dev) return;
#pragma unroll
    for (int o = 0; o < D; ++o) sc[o][threadIdx.x] = 0;
    int32_t g[D + 1];
    load_grid<D>(gv, c, g);
    const int dk = gv.b.inst[g[0]].d;
    auto emit = [&](uint32_t a, int o) {
        if (a != (uint32_t)c) sc[o][threadIdx.x] += 1;
    };
    query<D>(t, g, dk, emit);
#pragma unroll
    for (int o = 0; o < D; ++o) off_counts[c * D + o] = sc[o][threadIdx.x];
}

template <int D>
__global__ __launch_bounds__(kBlock) void nei_fill_kernel(GridView gv, TreeView t, const uint32_t* __restrict__ off_counts,
                                                          const uint64_t* __restrict__ nei_off, uint32_t* __restrict__ nei,
                                                          uint64_t capacity) {
    __shared__ uint32_t pos[D][kBlock];
    const int64_t ncell = *gv.ncell_dev;
    if (nei_off[ncell] > capacity) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&gv.b.hdr->err, kErrNeiOverflow);
        return;
    }
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncell) return;
    uint32_t acc = 0;
#pragma unroll
    for (int o = 0; o < D; ++o) {
        pos[o][threadIdx.x] = acc;
        acc += off_counts[c * D + o];
    }
    const uint64_t base = nei_off[c];
    int32_t g[D + 1];
    load_grid<D>(gv, c, g);
    const int dk = gv.b.inst[g[0]].d;
    auto emit = [&](uint32_t a, int o) {
        if (a != (uint32_t)c) {
            const uint32_t k = pos[o][threadIdx.x];
            pos[o][threadIdx.x] = k + 1;
            nei[base + k] = a;
        }
    };
    query<D>(t, g, dk, emit);
}

hipError_t launch_nei_count(const GridView& g, const TreeView& t, uint32_t* off_counts, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    GD_DISPATCH_D(g.D, (nei_count_kernel<D><<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(g, t, off_counts)));
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

__global__ void nei_total_kernel(const uint64_t* nei_off, const uint32_t* ncell, uint64_t* total) {
    *total = nei_off[*ncell];
}

hipError_t launch_nei_offsets(const GridView& g, const uint32_t* off_counts, uint64_t* nei_off, uint64_t* partial,
                              hipStream_t st) {
    // nei_off[c] for c in [0, ncell]; entries beyond the true ncell repeat the total
    hipError_t e = scan_exclusive<uint64_t>(CellTotal{off_counts, g.ncell_dev, g.D}, g.ncell + 1, nei_off,
                                            (uint64_t*)nullptr, partial, st);
    if (e != hipSuccess) return e;
    nei_total_kernel<<<1, 1, 0, st>>>(nei_off, g.ncell_dev, &g.b.hdr->nei_total);
    return hipGetLastError();
}

hipError_t launch_nei_fill(const GridView& g, const TreeView& t, const uint32_t* off_counts, const uint64_t* nei_off,
                           uint32_t* nei, uint64_t capacity, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    GD_DISPATCH_D(g.D, (nei_fill_kernel<D><<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(g, t, off_counts,
                                                                                               nei_off, nei, capacity)));
    return hipGetLastError();
}

}  // namespace gd
