// Device-wide exclusive prefix sum (reduce, scan of block totals, scan):
// three launches, no inter-workgroup waiting.  The input is a functor
// f(i) -> T so that flags can be formed on the fly from other arrays.
#pragma once

#include "common.hpp"

namespace gd {

constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;  // 4096 elements per workgroup

inline int64_t scan_blocks(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

template <typename T, typename F>
__global__ __launch_bounds__(kBlock) void scan_reduce_kernel(F f, int64_t n, T* partial) {
    __shared__ T wsum[kWavesPerBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    T s = 0;
#pragma unroll 4
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
        if (i < n) s += f(i);
    }
    s = wave_sum(s);
    if (lane_id() == 0) wsum[wave_id()] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) t += wsum[w];
        partial[blockIdx.x] = t;
    }
}

// One workgroup: exclusive scan of the block totals in place; grand total out.
template <typename T>
__global__ __launch_bounds__(kBlock) void scan_partials_kernel(T* partial, int64_t nb, T* total) {
    __shared__ T wsum[kWavesPerBlock];
    T carry = 0;
    for (int64_t base = 0; base < nb; base += kBlock) {
        const int64_t i = base + threadIdx.x;
        T v = i < nb ? partial[i] : T(0);
        T tot;
        T ex = block_excl_scan(v, wsum, tot);
        if (i < nb) partial[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <typename T, typename F>
__global__ __launch_bounds__(kBlock) void scan_down_kernel(F f, int64_t n, const T* partial, T* out) {
    __shared__ T wsum[kWavesPerBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    T carry = partial[blockIdx.x];
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
        if (base + (int64_t)r * kBlock >= n) break;  // uniform across the block
        T v = i < n ? f(i) : T(0);
        T tot;
        T ex = block_excl_scan(v, wsum, tot);
        if (i < n) out[i] = carry + ex;
        carry += tot;
    }
}

// out[i] = sum_{k < i} f(k) for 0 <= i < n; *total = sum of all (device).
// `partial` needs scan_blocks(n) elements.
template <typename T, typename F>
hipError_t scan_exclusive(F f, int64_t n, T* out, T* total, T* partial, hipStream_t st) {
    const int64_t nb = scan_blocks(n);
    if (nb == 0) {
        return total ? fill<T>(total, 1, T(0), st) : hipSuccess;
    }
    scan_reduce_kernel<T, F><<<dim3((unsigned)nb), dim3(kBlock), 0, st>>>(f, n, partial);
    scan_partials_kernel<T><<<1, kBlock, 0, st>>>(partial, nb, total);
    scan_down_kernel<T, F><<<dim3((unsigned)nb), dim3(kBlock), 0, st>>>(f, n, partial, out);
    return hipGetLastError();
}

template <typename T>
struct ArrayInput {
    const T* a;
    __device__ T operator()(int64_t i) const { return a[i]; }
};

}  // namespace gd
