// Non-empty neighbouring grids query (Section 4.2.2, Algorithm 3, Eq. (2)).
//
// One thread per grid g walks the grid tree level by level.  At level l it
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

template <int D, int L, typename Emit>
__device__ __forceinline__ void walk(const TreeView& t, const int32_t (&g)[D], uint32_t lo, uint32_t hi, int off,
                                     Emit& emit) {
    const int R = D - off;  // budget left, >= 1
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
        const int32_t dk = key[a] - g[L];
        if (dk > win) break;
        const int gap = (dk < 0 ? -dk : dk) - 1;
        const int o = off + (gap > 0 ? gap * gap : 0);
        if (o >= D) continue;
        if constexpr (L == D - 1) {
            emit(a, o);
        } else {
            walk<D, L + 1>(t, g, t.child[L][a], t.child[L][a + 1], o, emit);
        }
    }
}

template <int D>
__device__ __forceinline__ void load_grid(const GridView& gv, int64_t c, int32_t (&g)[D]) {
#pragma unroll
    for (int j = 0; j < D; ++j) g[j] = gv.ck[(int64_t)j * gv.ck_stride + c];
}

template <int D>
__global__ __launch_bounds__(kBlock) void nei_count_kernel(GridView gv, TreeView t, uint32_t* __restrict__ off_counts) {
    __shared__ uint32_t sc[D][kBlock];
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= gv.ncell) return;
#pragma unroll
    for (int o = 0; o < D; ++o) sc[o][threadIdx.x] = 0;
    int32_t g[D];
    load_grid<D>(gv, c, g);
    auto emit = [&](uint32_t a, int o) {
        if (a != (uint32_t)c) sc[o][threadIdx.x] += 1;
    };
    walk<D, 0>(t, g, 0u, t.level_count[0], 0, emit);
#pragma unroll
    for (int o = 0; o < D; ++o) off_counts[c * D + o] = sc[o][threadIdx.x];
}

template <int D>
__global__ __launch_bounds__(kBlock) void nei_fill_kernel(GridView gv, TreeView t, const uint32_t* __restrict__ off_counts,
                                                          const uint64_t* __restrict__ nei_off, uint32_t* __restrict__ nei) {
    __shared__ uint32_t pos[D][kBlock];
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= gv.ncell) return;
    uint32_t acc = 0;
#pragma unroll
    for (int o = 0; o < D; ++o) {
        pos[o][threadIdx.x] = acc;
        acc += off_counts[c * D + o];
    }
    const uint64_t base = nei_off[c];
    int32_t g[D];
    load_grid<D>(gv, c, g);
    auto emit = [&](uint32_t a, int o) {
        if (a != (uint32_t)c) {
            const uint32_t k = pos[o][threadIdx.x];
            pos[o][threadIdx.x] = k + 1;
            nei[base + k] = a;
        }
    };
    walk<D, 0>(t, g, 0u, t.level_count[0], 0, emit);
}

hipError_t launch_nei_count(const GridView& g, const TreeView& t, uint32_t* off_counts, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    GD_DISPATCH_D(g.d, (nei_count_kernel<D><<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(g, t, off_counts)));
    return hipGetLastError();
}

struct CellTotal {
    const uint32_t* oc;
    int64_t ncell;
    int d;
    __device__ uint64_t operator()(int64_t c) const {
        if (c >= ncell) return 0;
        uint64_t s = 0;
        for (int o = 0; o < d; ++o) s += oc[c * d + o];
        return s;
    }
};

hipError_t launch_nei_offsets(const GridView& g, const uint32_t* off_counts, uint64_t* nei_off, uint64_t* partial,
                              hipStream_t st) {
    // nei_off[ncell] receives the total
    return scan_exclusive<uint64_t>(CellTotal{off_counts, g.ncell, g.d}, g.ncell + 1, nei_off, (uint64_t*)nullptr,
                                    partial, st);
}

hipError_t launch_nei_fill(const GridView& g, const TreeView& t, const uint32_t* off_counts, const uint64_t* nei_off,
                           uint32_t* nei, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    GD_DISPATCH_D(g.d, (nei_fill_kernel<D><<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(g, t, off_counts,
                                                                                               nei_off, nei)));
    return hipGetLastError();
}

}  // namespace gd
