// Partitioning (Section 4.1, Algorithm 1) and the grid tree (Section 4.2.1,
// Algorithm 2) on gfx950.
//
//   minmax  : mn_j = min over P (Eq. (1)) and the input check (integers,
//             |x| <= 2^24), one pass with LDS + device atomics
//   keys    : identifiers of Eq. (1), exact (see grid_coord), packed into one
//             integer with dimension 1 in the highest bits, so that integer
//             order is the lexicographic order the paper's radix sort makes
//   gather  : sorted points as d separate int32 arrays (SoA) for coalesced
//             loads in the later phases
//   cells   : runs of equal identifiers = the non-empty grids Gs
//   tree    : one level per dimension; level l holds the distinct identifier
//             prefixes of length l+1 in sorted order, so every node's
//             children are contiguous and its child keys ascend
#include <climits>

#include "launch.hpp"
#include "scan.hpp"

namespace gd {

__global__ __launch_bounds__(kBlock) void minmax_kernel(const float* __restrict__ x, int64_t n, int d, int* mn,
                                                        int* mx, uint32_t* err) {
    __shared__ int smn[kMaxD], smx[kMaxD];
    if (threadIdx.x < kMaxD) {
        smn[threadIdx.x] = INT_MAX;
        smx[threadIdx.x] = INT_MIN;
    }
    __syncthreads();
    int lmn[kMaxD], lmx[kMaxD];
#pragma unroll
    for (int j = 0; j < kMaxD; ++j) {
        lmn[j] = INT_MAX;
        lmx[j] = INT_MIN;
    }
    bool bad = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
#pragma unroll
        for (int j = 0; j < kMaxD; ++j) {
            if (j < d) {
                const float v = x[i * d + j];
                const bool ok = (v == rintf(v)) && fabsf(v) <= 16777216.0f;
                bad |= !ok;
                const int iv = ok ? (int)v : 0;
                lmn[j] = min(lmn[j], ok ? iv : INT_MAX);
                lmx[j] = max(lmx[j], ok ? iv : INT_MIN);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kMaxD; ++j) {
        if (j < d) {
            int a = lmn[j], b = lmx[j];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                a = min(a, __shfl_xor(a, o));
                b = max(b, __shfl_xor(b, o));
            }
            if (lane_id() == 0) {
                atomicMin(&smn[j], a);
                atomicMax(&smx[j], b);
            }
        }
    }
    if (bad) atomicOr(err, kErrNotInteger);
    __syncthreads();
    if (threadIdx.x < (unsigned)d) {
        atomicMin(&mn[threadIdx.x], smn[threadIdx.x]);
        atomicMax(&mx[threadIdx.x], smx[threadIdx.x]);
    }
}

hipError_t launch_minmax(const float* x, int64_t n, int d, int* mn, int* mx, uint32_t* err, hipStream_t st) {
    hipError_t e = fill<int>(mn, kMaxD, INT_MAX, st);
    if (e != hipSuccess) return e;
    if ((e = fill<int>(mx, kMaxD, INT_MIN, st)) != hipSuccess) return e;
    if ((e = fill<uint32_t>(err, 1, 0u, st)) != hipSuccess) return e;
    if (n == 0) return hipSuccess;
    int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 2048) blocks = 2048;
    minmax_kernel<<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(x, n, d, mn, mx, err);
    return hipGetLastError();
}

template <typename K>
__global__ __launch_bounds__(kBlock) void keys_kernel(const float* __restrict__ x, int64_t n, KeyParams kp,
                                                      K* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    K key = 0;
#pragma unroll
    for (int j = 0; j < kMaxD; ++j) {
        if (j < kp.d) {
            const int64_t u = (int64_t)(int)x[i * kp.d + j] - kp.mn[j];
            key |= (K)grid_coord(u, kp.d, kp.eps) << kp.shift[j];
        }
    }
    keys[i] = key;
}

template <typename K>
hipError_t launch_keys(const float* x, int64_t n, const KeyParams& kp, K* keys, hipStream_t st) {
    if (n == 0) return hipSuccess;
    keys_kernel<K><<<dim3(grid_for(n)), dim3(kBlock), 0, st>>>(x, n, kp, keys);
    return hipGetLastError();
}
template hipError_t launch_keys<uint32_t>(const float*, int64_t, const KeyParams&, uint32_t*, hipStream_t);
template hipError_t launch_keys<uint64_t>(const float*, int64_t, const KeyParams&, uint64_t*, hipStream_t);

__global__ __launch_bounds__(kBlock) void gather_kernel(const float* __restrict__ x, int64_t n, KeyParams kp,
                                                        const uint32_t* __restrict__ sidx, int32_t* __restrict__ crd) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const int64_t o = sidx[s];
#pragma unroll
    for (int j = 0; j < kMaxD; ++j)
        if (j < kp.d) crd[(int64_t)j * n + s] = (int)x[o * kp.d + j] - kp.mn[j];
}

hipError_t launch_gather(const float* x, int64_t n, const KeyParams& kp, const uint32_t* sidx, int32_t* crd,
                         hipStream_t st) {
    if (n == 0) return hipSuccess;
    gather_kernel<<<dim3(grid_for(n)), dim3(kBlock), 0, st>>>(x, n, kp, sidx, crd);
    return hipGetLastError();
}

template <typename K>
struct KeyChange {
    const K* k;
    int64_t n;
    __device__ uint32_t operator()(int64_t i) const { return i < n && (i == 0 || k[i] != k[i - 1]); }
};

template <typename K>
__global__ __launch_bounds__(kBlock) void cells_kernel(const K* __restrict__ skeys, int64_t n, KeyParams kp,
                                                       const uint32_t* __restrict__ excl, uint32_t* cell_start,
                                                       uint32_t* cell_of, int32_t* ck, int64_t ck_stride) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= n) return;
    const K key = skeys[s];
    const bool first = s == 0 || skeys[s - 1] != key;
    const uint32_t c = excl[s] + (first ? 1u : 0u) - 1u;
    if (cell_of) cell_of[s] = c;
    if (first) {
        cell_start[c] = (uint32_t)s;
#pragma unroll
        for (int j = 0; j < kMaxD; ++j) {
            if (j < kp.d) {
                const K mask = (kp.bits[j] >= (int)(8 * sizeof(K))) ? ~K(0) : ((K(1) << kp.bits[j]) - 1);
                ck[(int64_t)j * ck_stride + c] = (int32_t)((key >> kp.shift[j]) & mask);
            }
        }
    }
    if (s == n - 1) cell_start[c + 1] = (uint32_t)n;
}

template <typename K>
hipError_t launch_cells(const K* skeys, int64_t n, const KeyParams& kp, uint32_t* excl, uint32_t* partial,
                        uint32_t* ncell_dev, uint32_t* cell_start, uint32_t* cell_of, int32_t* ck, int64_t ck_stride,
                        hipStream_t st) {
    hipError_t e = scan_exclusive<uint32_t>(KeyChange<K>{skeys, n}, n, excl, ncell_dev, partial, st);
    if (e != hipSuccess || n == 0) return e;
    cells_kernel<K><<<dim3(grid_for(n)), dim3(kBlock), 0, st>>>(skeys, n, kp, excl, cell_start, cell_of, ck,
                                                                ck_stride);
    return hipGetLastError();
}
template hipError_t launch_cells<uint32_t>(const uint32_t*, int64_t, const KeyParams&, uint32_t*, uint32_t*,
                                           uint32_t*, uint32_t*, uint32_t*, int32_t*, int64_t, hipStream_t);
template hipError_t launch_cells<uint64_t>(const uint64_t*, int64_t, const KeyParams&, uint32_t*, uint32_t*,
                                           uint32_t*, uint32_t*, uint32_t*, int32_t*, int64_t, hipStream_t);

// A grid starts a new node at level l iff it differs from the previous grid
// in one of dimensions 0..l (grids are in lexicographic order).
struct LevelFlag {
    const int32_t* ck;
    int64_t stride, ncell;
    int d, l;
    __device__ uint32_t operator()(int64_t c) const {
        if (c >= ncell) return 0;
        if (c == 0) return 1;
        for (int j = 0; j <= l; ++j)
            if (ck[(int64_t)j * stride + c] != ck[(int64_t)j * stride + c - 1]) return 1;
        return 0;
    }
};

struct TreeBuild {
    int32_t* key[kMaxD];
    uint32_t* child[kMaxD];
    const uint32_t* excl[kMaxD];  // per level: nodes before grid c (c in [0, ncell])
};

__global__ __launch_bounds__(kBlock) void tree_kernel(const int32_t* __restrict__ ck, int64_t stride, int64_t ncell,
                                                      int d, TreeBuild tb) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c > ncell) return;
    for (int l = 0; l + 1 < d; ++l) {
        LevelFlag f{ck, stride, ncell, d, l};
        if (c == ncell || f(c)) {
            const uint32_t a = tb.excl[l][c];
            if (c < ncell) tb.key[l][a] = ck[(int64_t)l * stride + c];
            // children: the level-(l+1) node that starts at grid c; level d-1 nodes are the grids
            tb.child[l][a] = (l + 2 < d) ? tb.excl[l + 1][c] : (uint32_t)c;
        }
    }
}

hipError_t launch_tree(const GridView& g, const KeyParams& kp, uint32_t* level_excl, uint32_t* partial,
                       uint32_t* level_count_dev, int32_t* const* tkey, uint32_t* const* tchild, hipStream_t st) {
    const int d = g.d;
    const int64_t stride = g.ck_stride;
    TreeBuild tb{};
    hipError_t e;
    // level d-1 are the grids: ncell nodes
    if ((e = fill<uint32_t>(level_count_dev + (d - 1), 1, (uint32_t)g.ncell, st)) != hipSuccess) return e;
    for (int l = 0; l + 1 < d; ++l) {
        uint32_t* ex = level_excl + (int64_t)l * (g.ncell + 1);
        e = scan_exclusive<uint32_t>(LevelFlag{g.ck, stride, g.ncell, d, l}, g.ncell + 1, ex, level_count_dev + l,
                                     partial, st);
        if (e != hipSuccess) return e;
        tb.key[l] = tkey[l];
        tb.child[l] = tchild[l];
        tb.excl[l] = ex;
    }
    if (d == 1 || g.ncell == 0) return hipSuccess;
    tree_kernel<<<dim3(grid_for(g.ncell + 1)), dim3(kBlock), 0, st>>>(g.ck, stride, g.ncell, d, tb);
    (void)kp;
    return hipGetLastError();
}

}  // namespace gd
