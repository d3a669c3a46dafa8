// Device-wide exclusive prefix sum: a reduce pass and a scan pass, no
// inter-workgroup waiting.  The input is a functor
// f(i) -> T so that flags can be formed on the fly from other arrays.
#pragma once

#include "common.hpp"

namespace gd {

// Scans of more than kScanMid elements take 16 elements per thread (4096 per
// workgroup); shorter ones 4 (1024 per workgroup), so that a scan over the
// grids still spreads over enough workgroups to hide the load latency.
constexpr int kScanItemsBig = 16;
constexpr int kScanItemsMid = 4;
constexpr int64_t kScanMid = 1 << 21;

inline int scan_items(int64_t n) { return n > kScanMid ? kScanItemsBig : kScanItemsMid; }
inline int64_t scan_blocks(int64_t n) {
    const int64_t tile = (int64_t)kBlock * scan_items(n);
    return (n + tile - 1) / tile;
}
// Partials needed by any scan of at most n elements.
inline int64_t scan_partial_cap(int64_t n) {
    const int64_t mid = n < kScanMid ? n : kScanMid;
    return (mid + kBlock * kScanItemsMid - 1) / (kBlock * kScanItemsMid) + scan_blocks(n);
}

// f over the workgroup's tile, element base + r * kBlock + threadIdx.x in
// v[r] (0 past n): every load of the tile is issued before the first use.
template <int kItems, typename T, typename F>
__device__ __forceinline__ void scan_load(F& f, int64_t n, int64_t base, T (&v)[kItems]) {
    if (base + (int64_t)kBlock * kItems <= n) {
#pragma unroll
        for (int r = 0; r < kItems; ++r) v[r] = f(base + (int64_t)r * kBlock + threadIdx.x);
    } else {
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
            v[r] = i < n ? f(i) : T(0);
        }
    }
}

template <typename T, int kItems, typename F>
__global__ __launch_bounds__(kBlock) void scan_reduce_kernel(F f, int64_t n, T* partial) {
    __shared__ T wsum[kWavesPerBlock];
    T v[kItems];
    scan_load<kItems>(f, n, (int64_t)blockIdx.x * kBlock * kItems, v);
    T s = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) s += v[r];
    s = wave_sum(s);
    if (lane_id() == 0) wsum[wave_id()] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
#pragma unroll
        for (int w = 0; w < kWavesPerBlock; ++w) t += wsum[w];
        partial[blockIdx.x] = t;
    }
}

// Output of a scan: store the exclusive prefix (or hand it to a functor,
// which also gets the element's own value v = f(i)).
template <typename T>
struct StoreOut {
    T* out;
    __device__ void operator()(int64_t i, T ex, T) const { out[i] = ex; }
};

// Each workgroup sums the totals of the tiles before it (a few thousand
// values at most, from L2) instead of waiting for a separate pass to scan
// them; the last workgroup writes the grand total.  The tile is read with
// coalesced loads, transposed through LDS so that each thread scans kItems
// consecutive elements (one workgroup scan per tile), and transposed back
// for coalesced output.  LDS rows are kItems + 1 long so that neither
// direction conflicts on banks.
template <typename T, int kItems, typename F, typename O>
__global__ __launch_bounds__(kBlock) void scan_down_kernel(F f, int64_t n, const T* partial, O o, T* total) {
    constexpr int kRow = kItems + 1;
    __shared__ T tile[kBlock * kRow];
    __shared__ T wsum[kWavesPerBlock];
    const int t = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kBlock * kItems;
    T v[kItems];
    scan_load<kItems>(f, n, base, v);
    T acc[8] = {};
    for (int64_t b0 = t; b0 < (int64_t)blockIdx.x; b0 += 8 * kBlock) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t b = b0 + (int64_t)u * kBlock;
            if (b < (int64_t)blockIdx.x) acc[u] += partial[b];
        }
    }
    T carry = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) carry += acc[u];
    carry = wave_sum(carry);
    if (lane_id() == 0) wsum[wave_id()] = carry;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int p = r * kBlock + t;
        tile[(p / kItems) * kRow + p % kItems] = v[r];
    }
    __syncthreads();
    carry = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) carry += wsum[w];
    T loc[kItems];
    T run = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        loc[k] = run;
        run += tile[t * kRow + k];
    }
    __syncthreads();  // wsum is reused by the workgroup scan
    T tot;
    const T ex = carry + block_excl_scan(run, wsum, tot);
#pragma unroll
    for (int k = 0; k < kItems; ++k) tile[t * kRow + k] = ex + loc[k];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int p = r * kBlock + t;
        const int64_t i = base + p;
        if (i < n) o(i, tile[(p / kItems) * kRow + p % kItems], v[r]);
    }
    if (total && blockIdx.x == gridDim.x - 1 && t == 0) *total = carry + tot;
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
            if (i0 + k < n) o(i0 + k, acc, v[k]);
            acc += v[k];
        }
        carry += tot;
    }
    if (t == 0 && total) *total = carry;
}

// o(i, sum_{k < i} f(k)) for 0 <= i < n; *total = sum of all (device).
// `partial` needs scan_blocks(n) elements (scan_partial_cap(m) covers every n <= m).
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
    if (scan_items(n) == kScanItemsBig) {
        scan_reduce_kernel<T, kScanItemsBig, F><<<dim3((unsigned)nb), dim3(kBlock), 0, st>>>(f, n, partial);
        scan_down_kernel<T, kScanItemsBig, F, O><<<dim3((unsigned)nb), dim3(kBlock), 0, st>>>(f, n, partial, o, total);
    } else {
        scan_reduce_kernel<T, kScanItemsMid, F><<<dim3((unsigned)nb), dim3(kBlock), 0, st>>>(f, n, partial);
        scan_down_kernel<T, kScanItemsMid, F, O><<<dim3((unsigned)nb), dim3(kBlock), 0, st>>>(f, n, partial, o, total);
    }
    return hipGetLastError();
}

// Scans of 0/1 flags whose output only concerns the set flags: w(i, r) for
// every i with f(i) = 1, r = its rank among the set flags, then w.end(total)
// once.  The scan pass needs no LDS transpose and no workgroup scan: wave w
// of the workgroup takes the w-th quarter of the reduce pass's tile, 64
// consecutive elements per round, and one ballot per round ranks the lanes.
// The set flags of the wave are listed in LDS and handed out one per lane,
// so the writer's loads for different flags are in flight together (called
// in place, each set flag would wait for the previous one's stores).
template <int kItems, typename F, typename W>
__global__ __launch_bounds__(kBlock) void flag_down_kernel(F f, int64_t n, const uint32_t* partial, W wr,
                                                           uint32_t* total) {
    constexpr int kPerWave = kWave * kItems;
    __shared__ uint32_t wcnt[kWavesPerBlock], wcarry[kWavesPerBlock];
    __shared__ uint16_t list[kWavesPerBlock][kPerWave];
    const int t = threadIdx.x, w = wave_id(), lane = lane_id();
    const int64_t tile0 = (int64_t)blockIdx.x * kBlock * kItems;
    const int64_t base = tile0 + (int64_t)w * kPerWave + lane;
    uint32_t v[kItems];
    if (tile0 + (int64_t)kBlock * kItems <= n) {
#pragma unroll
        for (int r = 0; r < kItems; ++r) v[r] = f(base + (int64_t)r * kWave);
    } else {
#pragma unroll
        for (int r = 0; r < kItems; ++r) {
            const int64_t i = base + (int64_t)r * kWave;
            v[r] = i < n ? f(i) : 0u;
        }
    }
    uint32_t acc[8] = {};
    for (int64_t b0 = t; b0 < (int64_t)blockIdx.x; b0 += 8 * kBlock) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int64_t b = b0 + (int64_t)u * kBlock;
            if (b < (int64_t)blockIdx.x) acc[u] += partial[b];
        }
    }
    uint32_t carry = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) carry += acc[u];
    carry = wave_sum(carry);
    // rank within the wave's run; the run's set flags listed in order
    const uint64_t lt = lanemask_lt();
    uint32_t cnt = 0;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const uint64_t m = ballot(v[r] != 0u);
        if (v[r]) list[w][cnt + (uint32_t)popc64(m & lt)] = (uint16_t)(r * kWave + lane);
        cnt += (uint32_t)popc64(m);
    }
    if (lane == 0) {
        wcnt[w] = cnt;
        wcarry[w] = carry;
    }
    __syncthreads();
    uint32_t c = 0, before = 0, all = 0;
#pragma unroll
    for (int ww = 0; ww < kWavesPerBlock; ++ww) {
        c += wcarry[ww];
        before += ww < w ? wcnt[ww] : 0u;
        all += wcnt[ww];
    }
    const int64_t run0 = tile0 + (int64_t)w * kPerWave;
    for (uint32_t j = (uint32_t)lane; j < cnt; j += kWave) wr(run0 + list[w][j], c + before + j);
    if (blockIdx.x == gridDim.x - 1 && t == 0) {
        if (total) *total = c + all;
        wr.end(c + all);
    }
}

// The same writer on the general scan (short inputs): w for each set flag,
// w.end after the last element.
template <typename W>
struct FlagOut {
    W wr;
    int64_t n;
    __device__ void operator()(int64_t i, uint32_t ex, uint32_t v) const {
        if (v) wr(i, ex);
        if (i == n - 1) wr.end(ex + v);
    }
};

// Flag scan with a writer of the set flags (see flag_down_kernel); with
// n = 0 the writer is not called.
template <typename F, typename W>
hipError_t scan_flags_apply(F f, int64_t n, W wr, uint32_t* total, uint32_t* partial, hipStream_t st) {
    const int64_t nb = scan_blocks(n);
    if (nb == 0 || n <= kSingleScanMax) return scan_apply<uint32_t>(f, n, FlagOut<W>{wr, n}, total, partial, st);
    if (scan_items(n) == kScanItemsBig) {
        scan_reduce_kernel<uint32_t, kScanItemsBig, F><<<dim3((unsigned)nb), dim3(kBlock), 0, st>>>(f, n, partial);
        flag_down_kernel<kScanItemsBig, F, W><<<dim3((unsigned)nb), dim3(kBlock), 0, st>>>(f, n, partial, wr, total);
    } else {
        scan_reduce_kernel<uint32_t, kScanItemsMid, F><<<dim3((unsigned)nb), dim3(kBlock), 0, st>>>(f, n, partial);
        flag_down_kernel<kScanItemsMid, F, W><<<dim3((unsigned)nb), dim3(kBlock), 0, st>>>(f, n, partial, wr, total);
    }
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
