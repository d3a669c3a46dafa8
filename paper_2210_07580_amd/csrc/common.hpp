// Shared device helpers for the gfx950 kernels: wave64 primitives, exact
// integer helpers and the launch-side error type.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.hpp"

namespace gd {

constexpr int kWave = 64;
constexpr int kBlock = 256;                 // 4 waves per workgroup
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr uint32_t kNone = 0xFFFFFFFFu;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
// The wave's index in its workgroup, visibly uniform (per-wave values derived
// from it stay in scalar registers).
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }
__device__ __forceinline__ uint64_t ballot(bool p) { return (uint64_t)__ballot(p); }
__device__ __forceinline__ int popc64(uint64_t m) { return __popcll(m); }
// index of the lowest set bit (m != 0)
__device__ __forceinline__ int ffs64(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }

// Pointers read from device-side tables (an instance's input and output
// arrays) are generic to the compiler, which then emits flat instructions
// (they also wait on the LDS counter); those arrays always live in global
// memory, so the point kernels say so.
#define GD_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T GD_GLOBAL* as_global(T* p) {
    return (T GD_GLOBAL*)p;
}

// Packed grid identifiers wider than 64 bits (d dimensions of up to ~18
// bits each): two words, with the few operators the identifier, sort and
// grid-run code applies to its key type.
struct Key128 {
    uint64_t lo, hi;
    Key128() = default;
    __host__ __device__ constexpr Key128(uint64_t v) : lo(v), hi(0) {}
    __host__ __device__ constexpr Key128(uint64_t l, uint64_t h) : lo(l), hi(h) {}
    __host__ __device__ friend bool operator==(const Key128& a, const Key128& b) { return a.lo == b.lo && a.hi == b.hi; }
    __host__ __device__ friend bool operator!=(const Key128& a, const Key128& b) { return !(a == b); }
    __host__ __device__ Key128 operator~() const { return Key128(~lo, ~hi); }
    __host__ __device__ Key128 operator|(const Key128& o) const { return Key128(lo | o.lo, hi | o.hi); }
    __host__ __device__ Key128 operator&(const Key128& o) const { return Key128(lo & o.lo, hi & o.hi); }
    __host__ __device__ Key128& operator|=(const Key128& o) {
        lo |= o.lo;
        hi |= o.hi;
        return *this;
    }
    __host__ __device__ Key128 operator<<(int s) const {
        if (s <= 0) return *this;
        if (s >= 128) return Key128(0, 0);
        if (s >= 64) return Key128(0, lo << (s - 64));
        return Key128(lo << s, (hi << s) | (lo >> (64 - s)));
    }
    __host__ __device__ Key128 operator>>(int s) const {
        if (s <= 0) return *this;
        if (s >= 128) return Key128(0, 0);
        if (s >= 64) return Key128(hi >> (s - 64), 0);
        return Key128((lo >> s) | (hi << (64 - s)), hi >> s);
    }
    __host__ __device__ explicit operator uint32_t() const { return (uint32_t)lo; }
    __host__ __device__ explicit operator uint64_t() const { return lo; }
};

// Field of `bits` bits at `shift` of a packed identifier (0 beyond its width).
template <typename K>
__host__ __device__ __forceinline__ uint64_t key_field(K key, int shift, int bits) {
    if (shift >= (int)(8 * sizeof(K))) return 0;
    const uint64_t v = (uint64_t)(key >> shift);
    return bits >= 64 ? v : (v & ((1ull << bits) - 1ull));
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)v);
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Orders LDS writes of a wave before its later LDS reads (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A 64-bit value that is the same in every lane, made visibly uniform so the
// compiler keeps it (and loops over its bits) in scalar registers.
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int32_t readlane(int32_t v, int lane) { return __builtin_amdgcn_readlane(v, lane); }
__device__ __forceinline__ uint32_t readlane(uint32_t v, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// Squared distance between points of neighbouring grids.  Every coordinate
// difference is below 2^24 and the sum below 9 eps^2 < 2^32, so 24-bit
// multiplies and a 32-bit sum are exact.
__device__ __forceinline__ uint32_t sq24(int32_t a, int32_t b) {
    const uint32_t t = (uint32_t)(a > b ? a - b : b - a);
    return __umul24(t, t);
}

// Squared distances of the wide path (eps above the 32-bit bound): any two
// points differ by less than 2^25 per coordinate, so each square is below
// 2^50 and a sum over at most eight coordinates below 2^53, exact in 64 bits.
template <bool kWide>
__device__ __forceinline__ typename Dist<kWide>::T sqd(int32_t a, int32_t b) {
    if constexpr (kWide) {
        const int64_t t = (int64_t)a - (int64_t)b;
        return (uint64_t)(t * t);
    } else {
        return sq24(a, b);
    }
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t t = __shfl_xor(v, o);
        v = t > v ? t : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint64_t t = __shfl_xor(v, o);
        v = t < v ? t : v;
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        uint32_t t = __shfl_xor(v, o);
        v = t < v ? t : v;
    }
    return v;
}

// inclusive prefix sum across the 64 lanes
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T t = __shfl_up(v, o);
        if (l >= o) v += t;
    }
    return v;
}

// Exclusive prefix sum over a 256-thread block; `wsum` is 4 slots of shared
// memory.  Every thread of the block must call it.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* wsum, T& total) {
    T incl = wave_incl_scan(v);
    if (lane_id() == kWave - 1) wsum[wave_id()] = incl;
    __syncthreads();
    T off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) {
        T s = wsum[w];
        off += (w < wave_id()) ? s : T(0);
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + incl - v;
}

// Coherent (device-scope) access for data other workgroups update
// concurrently, such as union-find parents.
template <typename T>
__device__ __forceinline__ T load_acq(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_rel(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// floor(u * sqrt(d) / eps) exactly, for integers 0 <= u <= 2^25, 1 <= d <= 8,
// 1 <= eps < 2^15: the largest k with (k * eps)^2 <= d * u^2.  A float
// estimate (scale = sqrt(d) / eps) is corrected by exact 64-bit integer
// tests; d * u^2 < 2^54 and k * eps stays below 2^32.
__device__ __forceinline__ uint32_t grid_coord(uint32_t u, uint32_t d, uint32_t eps, float scale) {
    const uint64_t y = (uint64_t)(d * u) * u;
    uint32_t k = (uint32_t)((float)u * scale);
    for (;;) {
        const uint64_t ke = (uint64_t)k * eps;
        if (k == 0 || ke * ke <= y) break;
        --k;
    }
    for (;;) {
        const uint64_t ke = (uint64_t)(k + 1) * eps;
        if (ke * ke > y) break;
        ++k;
    }
    return k;
}

// Point rows: the coordinates of a point as one padded record of
// row_stride(D) int32 (1, 2, 4 or 8), so that one vector load fetches it.
constexpr int row_stride(int D) { return D <= 1 ? 1 : D == 2 ? 2 : D <= 4 ? 4 : 8; }

template <int D>
__device__ __forceinline__ void load_row(const int32_t* __restrict__ rows, int64_t r, int32_t (&y)[D]) {
    constexpr int S = row_stride(D);
    if constexpr (S == 1) {
        y[0] = rows[r];
    } else if constexpr (S == 2) {
        const int2 t = reinterpret_cast<const int2*>(rows)[r];
        y[0] = t.x;
        y[1] = t.y;
    } else if constexpr (S == 4) {
        const int4 t = reinterpret_cast<const int4*>(rows)[r];
        const int32_t v[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int k = 0; k < D; ++k) y[k] = v[k];
    } else {
        const int4 a = reinterpret_cast<const int4*>(rows)[2 * r];
        const int4 b = reinterpret_cast<const int4*>(rows)[2 * r + 1];
        const int32_t v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
        for (int k = 0; k < D; ++k) y[k] = v[k];
    }
}

// Store a row; the padding is written as 0.
template <int D>
__device__ __forceinline__ void store_row(int32_t* __restrict__ rows, int64_t r, const int32_t (&y)[D]) {
    constexpr int S = row_stride(D);
    int32_t v[S];
#pragma unroll
    for (int k = 0; k < S; ++k) v[k] = k < D ? y[k < D ? k : 0] : 0;
    if constexpr (S == 1) {
        rows[r] = v[0];
    } else if constexpr (S == 2) {
        reinterpret_cast<int2*>(rows)[r] = make_int2(v[0], v[1]);
    } else if constexpr (S == 4) {
        reinterpret_cast<int4*>(rows)[r] = make_int4(v[0], v[1], v[2], v[3]);
    } else {
        reinterpret_cast<int4*>(rows)[2 * r] = make_int4(v[0], v[1], v[2], v[3]);
        reinterpret_cast<int4*>(rows)[2 * r + 1] = make_int4(v[4], v[5], v[6], v[7]);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void fill_kernel(T* p, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        p[i] = v;
}

// Fill with a kernel rather than a memset node, so that the sequence can be
// captured into a HIP graph.
template <typename T>
inline hipError_t fill(T* p, int64_t n, T v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    fill_kernel<T><<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(p, n, v);
    return hipGetLastError();
}

// Workgroups are handed to the 8 XCDs of the chip round robin by index, and
// each XCD has its own L2.  xcd_order(b, count) is the work item that
// workgroup b takes so that every XCD walks one contiguous range of items in
// order (a bijection of [0, count); only the speed depends on it).  Kernels
// whose neighbouring items share data (neighbouring grids read largely the
// same neighbour rows and tree nodes) then find it in their own L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t count) {
    const int64_t q = count / kXcds, r = count % kXcds;
    const int64_t x = b % kXcds, j = b / kXcds;
    return x * q + (x < r ? x : r) + j;
}

// The same in runs of kRun items: XCD x takes runs x, x + 8, x + 16, ...
// (locality within a run, every XCD spread over the whole range so that
// uneven work is shared); the items past the last full group of 8 runs keep
// their own index.
template <int kRun>
__device__ __forceinline__ int64_t xcd_runs(int64_t b, int64_t count) {
    constexpr int64_t kGroup = (int64_t)kXcds * kRun;
    if (b >= count / kGroup * kGroup) return b;
    const int64_t x = b % kXcds, j = b / kXcds;
    return (j / kRun) * kGroup + x * kRun + j % kRun;
}

// Whether some query of `open` (lanes of the wave, rows qx: x - mn) lies within eps
// of grid cc's cell: coordinate j of the cell spans [g_j s, (g_j + 1) s)
// with s = eps / sqrt(d) (Eq. (1)).  Conservative: lim is eps^2 widened
// beyond the rounding of the cell bounds, so a grid is only dropped when no
// point of it can be within eps of any query.
template <int D>
__device__ __forceinline__ bool cell_near(const GridView& gv, uint32_t cc, uint64_t open, const int32_t (&qx)[D],
                                          double side, double lim) {
    double lo[D];
#pragma unroll
    for (int j = 0; j < D; ++j) lo[j] = (double)gv.ck[(int64_t)(j + 1) * gv.ck_stride + cc] * side;
    bool near = false;
    for (uint64_t m = open; m; m &= m - 1ull) {
        const int qi = ffs64(m);
        double d2 = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double q = (double)readlane(qx[j], qi);
            const double g = q < lo[j] ? lo[j] - q : (q > lo[j] + side ? q - lo[j] - side : 0.0);
            d2 += g * g;
        }
        near |= d2 <= lim;
    }
    return near;
}

#define GD_DISPATCH_D(d, CALL)                             \
    do {                                                   \
        switch (d) {                                       \
            case 1: { constexpr int D = 1; CALL; } break;  \
            case 2: { constexpr int D = 2; CALL; } break;  \
            case 3: { constexpr int D = 3; CALL; } break;  \
            case 4: { constexpr int D = 4; CALL; } break;  \
            case 5: { constexpr int D = 5; CALL; } break;  \
            case 6: { constexpr int D = 6; CALL; } break;  \
            case 7: { constexpr int D = 7; CALL; } break;  \
            case 8: { constexpr int D = 8; CALL; } break;  \
            default: return hipErrorInvalidValue;          \
        }                                                  \
    } while (0)

inline unsigned grid_for(int64_t n, int per_block = kBlock) {
    int64_t b = (n + per_block - 1) / per_block;
    return (unsigned)(b < 1 ? 1 : b);
}

// A dispatch counts its work-items in 32 bits per grid dimension: a grid of
// 2^32 work-items or more in x wraps silently and runs only the remainder.
// Kernels with several lanes per grid (a wave per grid reaches that bound at
// 2^26 grids) are launched with grid_of(): at most 2^21 workgroups (of at most
// 1024 lanes) in x, the rest as rows in y, and they number their workgroups
// with block_id() / block_count(), which are blockIdx.x / gridDim.x whenever
// y is 1.  The last row may hold workgroups past the count asked for; the
// kernels' range checks drop them.
constexpr int64_t kMaxGridX = int64_t(1) << 21;
inline dim3 grid_of(int64_t blocks) {
    if (blocks <= kMaxGridX) return dim3((unsigned)(blocks < 1 ? 1 : blocks));
    return dim3((unsigned)kMaxGridX, (unsigned)((blocks + kMaxGridX - 1) / kMaxGridX));
}
__device__ __forceinline__ int64_t block_id() { return (int64_t)blockIdx.y * gridDim.x + blockIdx.x; }
__device__ __forceinline__ int64_t block_count() { return (int64_t)gridDim.y * gridDim.x; }

}  // namespace gd
