// Device-wide exclusive prefix sum: a reduce pass and a scan pass, no
// inter-workgroup waiting.  The input is a functor
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

// Output of a scan: store the exclusive prefix (or hand it to a functor).
template <typename T>
struct StoreOut {
    T* out;
    __device__ void operator()(int64_t i, T ex) const { out[i] = ex; }
};

// Each workgroup sums the totals of the tiles before it (a few thousand
// values at most, from L2) instead of waiting for a separate pass to scan
// them; the last workgroup writes the grand total.
template <typename T, typename F, typename O>
__global__ __launch_bounds__(kBlock) void scan_down_kernel(F f, int64_t n, const T* partial, O o, T* total) {
    __shared__ T wsum[kWavesPerBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    T carry = 0;
    for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += kBlock) carry += partial[b];
    carry = wave_sum(carry);
    if (lane_id() == 0) wsum[wave_id()] = carry;
    __syncthreads();
    carry = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) carry += wsum[w];
    __syncthreads();
    for (int r = 0; r < kScanItems; ++r) {
        const int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
        if (base + (int64_t)r * kBlock >= n) break;  // uniform across the block
        T v = i < n ? f(i) : T(0);
        T tot;
        T ex = block_excl_scan(v, wsum, tot);
        if (i < n) o(i, carry + ex);
        carry += tot;
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = carry;
}

// Short scans (up to kSingleScanMax elements) run in one workgroup of 1024
// threads: rounds of 4096 elements, four consecutive ones per thread, one
// workgroup scan per round.  One launch instead of three.
constexpr int kSingleScanThreads = 1024;
constexpr int64_t kSingleScanMax = 1 << 13;  // above this, three launches over many workgroups are faster

template <typename T, typename F, typename O>
__global__ __launch_bounds__(kSingleScanThreads) void scan_single_kernel(F f, int64_t n, O o, T* total) {
    constexpr int kW = kSingleScanThreads / kWave;
    __shared__ T wsum[kW];
    const int t = threadIdx.x, lane = lane_id(), w = wave_id();
    T carry = 0;
    for (int64_t base = 0; base < n; base += 4 * kSingleScanThreads) {
        const int64_t i0 = base + 4 * (int64_t)t;
        T v[4];
        T run = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = i0 + k < n ? f(i0 + k) : T(0);
            run += v[k];
        }
        const T incl = wave_incl_scan(run);
        if (lane == kWave - 1) wsum[w] = incl;
        __syncthreads();
        T off = 0, tot = 0;
#pragma unroll
        for (int ww = 0; ww < kW; ++ww) {
            const T x = wsum[ww];
            off += ww < w ? x : T(0);
            tot += x;
        }
        __syncthreads();
        T acc = carry + off + incl - run;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (i0 + k < n) o(i0 + k, acc);
            acc += v[k];
        }
        carry += tot;
    }
    if (t == 0 && total) *total = carry;
}

// o(i, sum_{k < i} f(k)) for 0 <= i < n; *total = sum of all (device).
// `partial` needs scan_blocks(n) elements.
template <typename T, typename F, typename O>
hipError_t scan_apply(F f, int64_t n, O o, T* total, T* partial, hipStream_t st) {
    const int64_t nb = scan_blocks(n);
    if (nb == 0) {
        return total ? fill<T>(total, 1, T(0), st) : hipSuccess;
    }
    if (n <= kSingleScanMax) {
        scan_single_kernel<T, F, O><<<1, kSingleScanThreads, 0, st>>>(f, n, o, total);
        return hipGetLastError();
    }
    scan_reduce_kernel<T, F><<<dim3((unsigned)nb), dim3(kBlock), 0, st>>>(f, n, partial);
    scan_down_kernel<T, F, O><<<dim3((unsigned)nb), dim3(kBlock), 0, st>>>(f, n, partial, o, total);
    return hipGetLastError();
}

// out[i] = sum_{k < i} f(k) for 0 <= i < n; *total = sum of all (device).
template <typename T, typename F>
hipError_t scan_exclusive(F f, int64_t n, T* out, T* total, T* partial, hipStream_t st) {
    return scan_apply<T>(f, n, StoreOut<T>{out}, total, partial, st);
}

template <typename T>
struct ArrayInput {
    const T* a;
    __device__ T operator()(int64_t i) const { return a[i]; }
};

}  // namespace gd
