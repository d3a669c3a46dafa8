// Partitioning (Section 4.1, Algorithm 1) and the grid tree (Section 4.2.1,
// Algorithm 2) on gfx950, for a batch of instances.
//
//   minmax  : mn_j = min over each instance's points (Eq. (1)) and the input
//             check (finite integers, |x| <= 2^24); one workgroup per point
//             tile leaves a record per tile, one workgroup per instance
//             folds them
//   layout  : per instance, the bit width of each identifier field; the
//             instance id goes above the widest instance's fields
//   keys    : identifiers of Eq. (1), exact (see grid_coord), packed into one
//             integer with the instance in the top field and dimension 1
//             highest below it, so integer order is the lexicographic order
//             the paper's radix sort produces, instance by instance
//   rows    : sorted points as padded int32 rows (one vector load per point
//             in the later phases; instances with d < D padded with 0),
//             rebuilt in sorted order from the low coordinate bits the sort
//             carried (unpack) or, when those do not fit, gathered
//   cells   : runs of equal identifiers = the non-empty grids Gs
//   tree    : level 0 = instances, level l = distinct prefixes of length l,
//             each level in sorted order, so every node's children are
//             contiguous and their keys ascend
#include <algorithm>
#include <type_traits>
#include <climits>

#include "launch.hpp"
#include "scan.hpp"

namespace gd {

// Visit the points [lo, hi) of instance I (lo a multiple of 4): each thread
// takes groups of four consecutive points, read as d float4 loads when the
// rows are 16-byte aligned (four rows of d floats span exactly d float4),
// then the remainder one point at a time.  f(i, row) gets the point index and
// its d coordinates.
// for_point_groups: the same walk, but each aligned group of four goes to
// fg(i0, rows) at once (so that its outputs can be stored as vectors) and
// only the remainder to f(i, row).
template <int D, typename FG, typename F>
__device__ __forceinline__ void for_point_groups(const Inst& I, int64_t lo, int64_t hi, FG&& fg, F&& f) {
    const float GD_GLOBAL* __restrict__ x = as_global(I.x);
    int64_t rest = lo;
    if ((reinterpret_cast<uintptr_t>(I.x) & 15u) == 0) {
        const int64_t groups = (hi - lo) >> 2;
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 GD_GLOBAL* __restrict__ xv = reinterpret_cast<const f4 GD_GLOBAL*>(x + lo * D);
#pragma unroll 2
        for (int64_t gi = threadIdx.x; gi < groups; gi += kBlock) {
            float v[4 * D];
#pragma unroll
            for (int q = 0; q < D; ++q) {
                const f4 t = xv[gi * D + q];
                v[4 * q + 0] = t.x;
                v[4 * q + 1] = t.y;
                v[4 * q + 2] = t.z;
                v[4 * q + 3] = t.w;
            }
            float rows[4][D];
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int j = 0; j < D; ++j) rows[p][j] = v[p * D + j];
            fg(lo + 4 * gi, rows);
        }
        rest = lo + 4 * groups;
    }
    for (int64_t i = rest + threadIdx.x; i < hi; i += kBlock) {
        float row[D];
#pragma unroll
        for (int j = 0; j < D; ++j) row[j] = x[i * D + j];
        f(i, row);
    }
}

template <int D, typename F>
__device__ __forceinline__ void for_points(const Inst& I, int64_t lo, int64_t hi, F&& f) {
    const float GD_GLOBAL* __restrict__ x = as_global(I.x);
    int64_t rest = lo;
    if ((reinterpret_cast<uintptr_t>(I.x) & 15u) == 0) {
        const int64_t groups = (hi - lo) >> 2;
        typedef float f4 __attribute__((ext_vector_type(4)));
        const f4 GD_GLOBAL* __restrict__ xv = reinterpret_cast<const f4 GD_GLOBAL*>(x + lo * D);
#pragma unroll 2
        for (int64_t gi = threadIdx.x; gi < groups; gi += kBlock) {
            float v[4 * D];
#pragma unroll
            for (int q = 0; q < D; ++q) {
                const f4 t = xv[gi * D + q];
                v[4 * q + 0] = t.x;
                v[4 * q + 1] = t.y;
                v[4 * q + 2] = t.z;
                v[4 * q + 3] = t.w;
            }
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                float row[D];
#pragma unroll
                for (int j = 0; j < D; ++j) row[j] = v[p * D + j];
                f(lo + 4 * gi + p, row);
            }
        }
        rest = lo + 4 * groups;
    }
    for (int64_t i = rest + threadIdx.x; i < hi; i += kBlock) {
        float row[D];
#pragma unroll
        for (int j = 0; j < D; ++j) row[j] = x[i * D + j];
        f(i, row);
    }
}

template <int D>
__device__ __forceinline__ void minmax_tile(Inst& I, int64_t lo, int64_t hi, int* smn, int* smx) {
    int lmn[D], lmx[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        lmn[j] = INT_MAX;
        lmx[j] = INT_MIN;
    }
    bool bad = false;
    for_points<D>(I, lo, hi, [&](int64_t, const float (&row)[D]) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const float v = row[j];
            const bool ok = (v == rintf(v)) && fabsf(v) <= 16777216.0f;
            bad |= !ok;
            lmn[j] = min(lmn[j], ok ? (int)v : INT_MAX);
            lmx[j] = max(lmx[j], ok ? (int)v : INT_MIN);
        }
    });
#pragma unroll
    for (int j = 0; j < D; ++j) {
        int a = lmn[j], c = lmx[j];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            a = min(a, __shfl_xor(a, o));
            c = max(c, __shfl_xor(c, o));
        }
        if (lane_id() == 0) {
            smn[wave_id() * kMaxD + j] = a;
            smx[wave_id() * kMaxD + j] = c;
        }
    }
    if (ballot(bad) && lane_id() == 0) atomicOr(&I.err, kErrNotInteger);
}

// Each workgroup leaves its tile's minima and maxima in part (one 64-byte
// record per tile, plain stores: a few thousand workgroups updating the same
// two words with device atomics serialise on them).
// Calls f(std::integral_constant<int, d>) for 1 <= d <= DB, the batch's
// largest dimension: a kernel compiled for DB holds registers for d <= DB
// only (one compiled for every d would size them all for d = 8).
template <int DB, int D = 1, typename F>
__device__ __forceinline__ void with_d(int d, F&& f) {
    if constexpr (D < DB) {
        if (d != D) {
            with_d<DB, D + 1>(d, f);
            return;
        }
    }
    f(std::integral_constant<int, D>{});
}

template <int DB>
__global__ __launch_bounds__(kBlock) void minmax_kernel(Batch b, int32_t* __restrict__ part) {
    constexpr int kWaves = kBlock / kWave;
    __shared__ int smn[kWaves * kMaxD], smx[kWaves * kMaxD];
    const int k = tile_instance(b, blockIdx.x);
    Inst& I = const_cast<Inst&>(b.inst[k]);
    const int d = I.d;
    const int64_t lo = (int64_t)(blockIdx.x - I.tile0) * b.tile_pts;
    const int64_t hi = min(I.n, lo + b.tile_pts);
    with_d<DB>(d, [&](auto dc) { minmax_tile<decltype(dc)::value>(I, lo, hi, smn, smx); });
    __syncthreads();
    if (threadIdx.x < (unsigned)d) {
        const int j = threadIdx.x;
        int a = smn[j], c = smx[j];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            a = min(a, smn[w * kMaxD + j]);
            c = max(c, smx[w * kMaxD + j]);
        }
        int32_t* rec = part + (int64_t)blockIdx.x * 2 * kMaxD;
        rec[j] = a;
        rec[kMaxD + j] = c;
    }
}

__device__ __forceinline__ int bit_length_u64(uint64_t v) { return v == 0 ? 0 : 64 - __clzll((long long)v); }

__device__ __forceinline__ uint64_t isqrt_u64(uint64_t y) {
    uint64_t r = (uint64_t)sqrt((double)y);
    while (r * r > y) --r;
    while ((r + 1) * (r + 1) <= y) ++r;
    return r;
}

// Field widths and shifts of instance I's identifiers from its minima and
// maxima; returns the identifier's bit count.  Everything is computed in
// registers and stored once at the end: reading a field back from memory
// would wait for the store before it.
__device__ int inst_layout(Inst& I, const int* mn, const int* mx) {
    const int d = I.d;
    const int64_t n = I.n;
    const uint64_t eps = (uint64_t)I.eps;
    int bits[kMaxD], shift[kMaxD];
    int total = 0;
#pragma unroll
    for (int j = 0; j < kMaxD; ++j) {
        bits[j] = 0;
        if (j < d) {
            const uint64_t u = n > 0 ? (uint64_t)((int64_t)mx[j] - mn[j]) : 0;
            bits[j] = bit_length_u64(isqrt_u64((uint64_t)d * u * u) / eps);
            total += bits[j];
        }
    }
    int sh = 0;
#pragma unroll
    for (int j = kMaxD - 1; j >= 0; --j) {
        shift[j] = sh;
        if (j < d) sh += bits[j];
    }
#pragma unroll
    for (int j = 0; j < kMaxD; ++j) {
        if (j < d) {
            I.bits[j] = bits[j];
            I.shift[j] = shift[j];
        }
    }
    I.key_bits = total;
    return total;
}

// Batch-wide layout: instance ids above the widest identifier.
__device__ void batch_layout(const Batch& b, int max_bits, uint32_t err, int plan_bits) {
    const int inst_bits = bit_length_u64((uint64_t)(b.count - 1));
    b.hdr->inst_shift = max_bits;
    b.hdr->total_bits = max_bits + inst_bits;
    if (max_bits + inst_bits > kMaxKeyBits) err |= kErrKeyBits;
    if (max_bits + inst_bits > plan_bits) err |= kErrPlan;
    b.hdr->err = err;
}

// One workgroup of 1024 threads per instance folds its tiles' records into mn
// and mx (a few thousand records: more threads, fewer dependent rounds).
// With kLayout (a batch of one instance) the same workgroup then lays out
// the identifiers, which saves the layout launch.
constexpr int kFinishThreads = 1024;
template <bool kLayout>
__global__ __launch_bounds__(kFinishThreads) void minmax_finish_kernel(Batch b, const int32_t* __restrict__ part,
                                                                       int plan_bits) {
    constexpr int kWaves = kFinishThreads / kWave;
    __shared__ int smn[kWaves * kMaxD], smx[kWaves * kMaxD];
    Inst& I = const_cast<Inst&>(b.inst[blockIdx.x]);
    const int d = I.d;
    const uint32_t nt = (uint32_t)((I.n + b.tile_pts - 1) / b.tile_pts);
    // thread t reads quarter q = t % 4 of records t / 4, t / 4 + 256, ...
    // (quarters 0-1: minima, 2-3: maxima), twelve records in flight: up to
    // 3072 tiles (12.5M points at 4096 per tile) in one round of loads
    const int q = threadIdx.x & 3;
    const bool is_min = q < 2;
    int4 acc = is_min ? make_int4(INT_MAX, INT_MAX, INT_MAX, INT_MAX) : make_int4(INT_MIN, INT_MIN, INT_MIN, INT_MIN);
    const int4* rec = reinterpret_cast<const int4*>(part + (int64_t)I.tile0 * 2 * kMaxD) + q;
    constexpr uint32_t kStep = kFinishThreads / 4;
    constexpr int kInFlight = 12;
    for (uint32_t t0 = threadIdx.x >> 2; t0 < nt; t0 += kInFlight * kStep) {
        int4 r[kInFlight];
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            const uint32_t t = t0 + u * kStep;
            r[u] = t < nt ? rec[(int64_t)t * 4] : acc;
        }
#pragma unroll
        for (int u = 0; u < kInFlight; ++u) {
            if (is_min) {
                acc.x = min(acc.x, r[u].x); acc.y = min(acc.y, r[u].y);
                acc.z = min(acc.z, r[u].z); acc.w = min(acc.w, r[u].w);
            } else {
                acc.x = max(acc.x, r[u].x); acc.y = max(acc.y, r[u].y);
                acc.z = max(acc.z, r[u].z); acc.w = max(acc.w, r[u].w);
            }
        }
    }
    // lanes with the same quarter: xor over 4, 8, 16, 32 keeps q
#pragma unroll
    for (int o = 4; o < kWave; o <<= 1) {
        const int4 b = make_int4(__shfl_xor(acc.x, o), __shfl_xor(acc.y, o), __shfl_xor(acc.z, o), __shfl_xor(acc.w, o));
        if (is_min) {
            acc.x = min(acc.x, b.x); acc.y = min(acc.y, b.y); acc.z = min(acc.z, b.z); acc.w = min(acc.w, b.w);
        } else {
            acc.x = max(acc.x, b.x); acc.y = max(acc.y, b.y); acc.z = max(acc.z, b.z); acc.w = max(acc.w, b.w);
        }
    }
    if (lane_id() < 4) {
        int* dst = (is_min ? smn : smx) + wave_id() * kMaxD + (q & 1) * 4;
        dst[0] = acc.x;
        dst[1] = acc.y;
        dst[2] = acc.z;
        dst[3] = acc.w;
    }
    __syncthreads();
    __shared__ int fmn[kMaxD], fmx[kMaxD];
    if (threadIdx.x < (unsigned)d) {
        const int j = threadIdx.x;
        int a = smn[j], c = smx[j];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            a = min(a, smn[w * kMaxD + j]);
            c = max(c, smx[w * kMaxD + j]);
        }
        I.mn[j] = a;
        I.mx[j] = c;
        fmn[j] = a;
        fmx[j] = c;
    }
    if constexpr (kLayout) {
        __syncthreads();
        if (threadIdx.x == 0) batch_layout(b, inst_layout(I, fmn, fmx), I.err, plan_bits);
    }
}

hipError_t launch_layout(const Batch& b, int plan_bits, hipStream_t st);

hipError_t launch_minmax(const Batch& b, int32_t* part, int plan_bits, hipStream_t st) {
    if (b.tiles == 0) return launch_layout(b, plan_bits, st);
    GD_DISPATCH_D(b.D, (minmax_kernel<D><<<dim3(b.tiles), dim3(kBlock), 0, st>>>(b, part)));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (b.count == 1) {
        minmax_finish_kernel<true><<<dim3(1), dim3(kFinishThreads), 0, st>>>(b, part, plan_bits);
        return hipGetLastError();
    }
    minmax_finish_kernel<false><<<dim3(b.count), dim3(kFinishThreads), 0, st>>>(b, part, plan_bits);
    const hipError_t e2 = hipGetLastError();
    if (e2 != hipSuccess) return e2;
    return launch_layout(b, plan_bits, st);
}

// One workgroup: per-instance field widths, then the batch-wide layout.
__global__ __launch_bounds__(kBlock) void layout_kernel(Batch b, int plan_bits) {
    __shared__ int s_max;
    __shared__ uint32_t s_err;
    if (threadIdx.x == 0) {
        s_max = 0;
        s_err = 0;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < b.count; k += kBlock) {
        Inst& I = const_cast<Inst&>(b.inst[k]);
        atomicMax(&s_max, inst_layout(I, I.mn, I.mx));
        if (I.err) atomicOr(&s_err, I.err);
    }
    __syncthreads();
    if (threadIdx.x == 0) batch_layout(b, s_max, s_err, plan_bits);
}

hipError_t launch_layout(const Batch& b, int plan_bits, hipStream_t st) {
    layout_kernel<<<1, kBlock, 0, st>>>(b, plan_bits);
    return hipGetLastError();
}

__global__ void plan_check_kernel(Header* h, int stage, int64_t cap_a, int64_t cap_b) {
    bool bad = (h->err & (kErrNotInteger | kErrKeyBits | kErrPlan)) != 0;
    if (stage == 0)
        bad |= (int64_t)h->ncell > cap_a;
    else if (stage == 1)
        bad |= h->nei_total > (uint64_t)cap_a;
    else
        bad |= (int64_t)h->counts[1] > cap_a || (int64_t)h->counts[2] > cap_b;
    if (bad) {
        h->err |= kErrPlan;
        h->ncell = 0;
        h->nei_total = 0;
        h->counts[1] = 0;
    }
}

hipError_t launch_plan_check(Header* hdr, int stage, int64_t cap_a, int64_t cap_b, hipStream_t st) {
    plan_check_kernel<<<1, 1, 0, st>>>(hdr, stage, cap_a, cap_b);
    return hipGetLastError();
}

// With `vals`, each point also gets the value that the sort carries for it:
// its index (low half) and the low pack_bits(d) bits of each coordinate
// (high half), from which unpack_kernel rebuilds the sorted rows.
template <int D, typename K>
__device__ __forceinline__ void keys_tile(const Inst& I, int64_t lo, int64_t hi, K top, K* __restrict__ keys,
                                          uint64_t* __restrict__ vals) {
    int32_t mn[D], sh[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        mn[j] = I.mn[j];
        sh[j] = I.shift[j];
    }
    const uint32_t eps = (uint32_t)I.eps;
    const float scale = (float)(sqrt((double)D) / (double)I.eps);
    constexpr int B = pack_bits(D);
    constexpr uint64_t kLow = B >= 32 ? 0xFFFFFFFFull : ((1ull << B) - 1ull);
    K* __restrict__ out = keys + I.off;
    auto point = [&](int64_t i, const float (&row)[D], K& key, uint64_t& val) {
        key = top;
        uint64_t packed = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const uint32_t u = (uint32_t)((int)row[j] - mn[j]);
            key |= (K)grid_coord(u, D, eps, scale) << sh[j];
            packed |= ((uint64_t)u & kLow) << (j * B);
        }
        val = (packed << 32) | (uint64_t)(uint32_t)(I.off + i);
    };
    // a group's four identifiers (and values) go out as 16-byte stores when
    // the instance starts on a multiple of four points
    const bool vec = (I.off & 3) == 0;
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    for_point_groups<D>(
        I, lo, hi,
        [&](int64_t i0, const float (&rows)[4][D]) {
            K kk[4];
            uint64_t vv[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) point(i0 + p, rows[p], kk[p], vv[p]);
            if (vec) {
                u4* ko = reinterpret_cast<u4*>(out + i0);
                if constexpr (sizeof(K) == 4) {
                    ko[0] = u4{(uint32_t)kk[0], (uint32_t)kk[1], (uint32_t)kk[2], (uint32_t)kk[3]};
                } else if constexpr (sizeof(K) == 8) {
                    ko[0] = u4{(uint32_t)kk[0], (uint32_t)((uint64_t)kk[0] >> 32), (uint32_t)kk[1],
                               (uint32_t)((uint64_t)kk[1] >> 32)};
                    ko[1] = u4{(uint32_t)kk[2], (uint32_t)((uint64_t)kk[2] >> 32), (uint32_t)kk[3],
                               (uint32_t)((uint64_t)kk[3] >> 32)};
                } else {
#pragma unroll
                    for (int p = 0; p < 4; ++p) out[i0 + p] = kk[p];  // one 16-byte store each
                }
                if (vals) {
                    u4* vo = reinterpret_cast<u4*>(vals + I.off + i0);
                    vo[0] = u4{(uint32_t)vv[0], (uint32_t)(vv[0] >> 32), (uint32_t)vv[1], (uint32_t)(vv[1] >> 32)};
                    vo[1] = u4{(uint32_t)vv[2], (uint32_t)(vv[2] >> 32), (uint32_t)vv[3], (uint32_t)(vv[3] >> 32)};
                }
            } else {
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    out[i0 + p] = kk[p];
                    if (vals) vals[I.off + i0 + p] = vv[p];
                }
            }
        },
        [&](int64_t i, const float (&row)[D]) {
            K key;
            uint64_t val;
            point(i, row, key, val);
            out[i] = key;
            if (vals) vals[I.off + i] = val;
        });
}

template <typename K, int DB>
__global__ __launch_bounds__(kBlock) void keys_kernel(Batch b, K* __restrict__ keys, uint64_t* __restrict__ vals) {
    const int k = tile_instance(b, blockIdx.x);
    const Inst& I = b.inst[k];
    const int64_t lo = (int64_t)(blockIdx.x - I.tile0) * b.tile_pts;
    const int64_t hi = min(I.n, lo + b.tile_pts);
    // a sync-free run whose instance table no longer allows packed rows (a
    // larger eps on replay) is discarded like one that outgrew its plan
    const bool bad_pack = vals && !pack_fits(I.d, I.eps);
    if (bad_pack && threadIdx.x == 0) atomicOr(&b.hdr->err, kErrPlan);
    if (bad_pack || (b.hdr->err & (kErrNotInteger | kErrKeyBits | kErrPlan))) {
        // a sync-free run on input it cannot handle (its result is discarded):
        // the instance id alone keeps every instance's points in its own
        // range through the sort, so later kernels stay within bounds
        for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
            keys[I.off + i] = (K)k;
            if (vals) vals[I.off + i] = (uint64_t)(uint32_t)(I.off + i);
        }
        return;
    }
    const int ishift = b.hdr->inst_shift;
    const K top = ishift >= (int)(8 * sizeof(K)) ? K(0) : (K)k << ishift;
    with_d<DB>(I.d, [&](auto dc) { keys_tile<decltype(dc)::value, K>(I, lo, hi, top, keys, vals); });
}

template <typename K>
hipError_t launch_keys(const Batch& b, K* keys, uint64_t* vals, hipStream_t st) {
    if (b.tiles == 0) return hipSuccess;
    GD_DISPATCH_D(b.D, (keys_kernel<K, D><<<dim3(b.tiles), dim3(kBlock), 0, st>>>(b, keys, vals)));
    return hipGetLastError();
}
template hipError_t launch_keys<uint32_t>(const Batch&, uint32_t*, uint64_t*, hipStream_t);
template hipError_t launch_keys<uint64_t>(const Batch&, uint64_t*, uint64_t*, hipStream_t);
template hipError_t launch_keys<Key128>(const Batch&, Key128*, uint64_t*, hipStream_t);

// Sorted rows without the random gather: the sort carried each point's
// index and the low B = pack_bits(d) bits of its coordinates u_j = x_j -
// mn_j.  The point's grid (from its sorted identifier) puts u_j in
// [g_j s, (g_j + 1) s) with s = eps / sqrt(d), so the grid's centre a_j is
// within s / 2 + 1 < 2^(B-1) of u_j (pack_fits), and u_j is the one value
// within 2^(B-1) of a_j with those low bits.  Reads and writes in sorted
// order only; tiles as the gather's.
template <int DB>
__global__ __launch_bounds__(kBlock) void unpack_kernel(Batch b, const uint32_t* __restrict__ skeys,
                                                        const uint64_t* __restrict__ vals,
                                                        uint32_t* __restrict__ sidx, int32_t* __restrict__ crd) {
    const int k = tile_instance(b, blockIdx.x);
    const Inst& I = b.inst[k];
    const int64_t lo = (int64_t)(blockIdx.x - I.tile0) * b.tile_pts;
    const int64_t hi = min(I.n, lo + b.tile_pts);
    with_d<DB>(I.d, [&](auto dc) {
        constexpr int D = decltype(dc)::value;
        constexpr int B = pack_bits(D);
        constexpr uint64_t kLow = B >= 32 ? 0xFFFFFFFFull : ((1ull << B) - 1ull);
        constexpr int64_t kHalf = (int64_t)1 << (B - 1);
        int sh[D];
        uint32_t fm[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            sh[j] = I.shift[j];
            fm[j] = I.bits[j] >= 32 ? 0xFFFFFFFFu : ((1u << I.bits[j]) - 1u);
        }
        const double side = (double)I.eps / sqrt((double)D);
#pragma unroll 4
        for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
            const int64_t s = I.off + i;
            const uint64_t v = vals[s];
            const uint32_t key = skeys[s];
            const uint64_t packed = v >> 32;
            int32_t y[DB];
#pragma unroll
            for (int j = 0; j < DB; ++j) y[j] = 0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const uint32_t g = (key >> sh[j]) & fm[j];
                const int64_t a = (int64_t)floor(((double)g + 0.5) * side);
                const uint64_t low = (packed >> (j * B)) & kLow;
                const uint64_t t = ((uint64_t)((int64_t)low - a + kHalf)) & kLow;
                y[j] = (int32_t)(a + (int64_t)t - kHalf);
            }
            store_row<DB>(crd, s, y);
            sidx[s] = (uint32_t)v;
        }
    });
}

hipError_t launch_unpack(const Batch& b, const uint32_t* skeys, const uint64_t* vals, uint32_t* sidx, int32_t* crd,
                         hipStream_t st) {
    if (b.tiles == 0) return hipSuccess;
    GD_DISPATCH_D(b.D, (unpack_kernel<D><<<dim3(b.tiles), dim3(kBlock), 0, st>>>(b, skeys, vals, sidx, crd)));
    return hipGetLastError();
}

// Packed rows in two-word keys (launch.hpp, pack64_bits): the word of a
// point is its identifier << W | its coordinates' low B bits (coordinate j at
// j * B), W = D * B for the batch's D.  Four points' words go out as two
// 16-byte stores when the instance starts on a multiple of four points.
template <int D>
__device__ __forceinline__ void keys64_tile(const Inst& I, int64_t lo, int64_t hi, uint64_t top, int B, int W,
                                            uint64_t* __restrict__ words) {
    int32_t mn[D], sh[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        mn[j] = I.mn[j];
        sh[j] = I.shift[j];
    }
    const uint32_t eps = (uint32_t)I.eps;
    const float scale = (float)(sqrt((double)D) / (double)I.eps);
    const uint64_t low = (1ull << B) - 1ull;
    uint64_t* __restrict__ out = words + I.off;
    auto point = [&](const float (&row)[D]) -> uint64_t {
        uint64_t key = top, packed = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const uint32_t u = (uint32_t)((int)row[j] - mn[j]);
            key |= (uint64_t)grid_coord(u, D, eps, scale) << sh[j];
            packed |= ((uint64_t)u & low) << (j * B);
        }
        return (key << W) | packed;
    };
    const bool vec = (I.off & 3) == 0;
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    for_point_groups<D>(
        I, lo, hi,
        [&](int64_t i0, const float (&rows)[4][D]) {
            uint64_t w[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) w[p] = point(rows[p]);
            if (vec) {
                u4* o = reinterpret_cast<u4*>(out + i0);
                o[0] = u4{(uint32_t)w[0], (uint32_t)(w[0] >> 32), (uint32_t)w[1], (uint32_t)(w[1] >> 32)};
                o[1] = u4{(uint32_t)w[2], (uint32_t)(w[2] >> 32), (uint32_t)w[3], (uint32_t)(w[3] >> 32)};
            } else {
#pragma unroll
                for (int p = 0; p < 4; ++p) out[i0 + p] = w[p];
            }
        },
        [&](int64_t i, const float (&row)[D]) { out[i] = point(row); });
}

template <int DB>
__global__ __launch_bounds__(kBlock) void keys64_kernel(Batch b, uint64_t* __restrict__ words, int B) {
    const int k = tile_instance(b, blockIdx.x);
    const Inst& I = b.inst[k];
    const int64_t lo = (int64_t)(blockIdx.x - I.tile0) * b.tile_pts;
    const int64_t hi = min(I.n, lo + b.tile_pts);
    const int W = b.D * B;
    // as keys_kernel: a sync-free run whose instances no longer fit B, or
    // whose input failed, is discarded; the instance id keeps each
    // instance's points in its own range through the sort
    const bool bad_pack = !pack_fits_bits(I.d, I.eps, B);
    if (bad_pack && threadIdx.x == 0) atomicOr(&b.hdr->err, kErrPlan);
    if (bad_pack || (b.hdr->err & (kErrNotInteger | kErrKeyBits | kErrPlan))) {
        for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) words[I.off + i] = (uint64_t)k << W;
        return;
    }
    const int ishift = b.hdr->inst_shift;
    const uint64_t top = ishift >= 64 ? 0ull : (uint64_t)k << ishift;
    with_d<DB>(I.d, [&](auto dc) { keys64_tile<decltype(dc)::value>(I, lo, hi, top, B, W, words); });
}

hipError_t launch_keys_packed64(const Batch& b, uint64_t* words, int bits, hipStream_t st) {
    if (b.tiles == 0) return hipSuccess;
    GD_DISPATCH_D(b.D, (keys64_kernel<D><<<dim3(b.tiles), dim3(kBlock), 0, st>>>(b, words, bits)));
    return hipGetLastError();
}

// The rows from the sorted words, as unpack_kernel does from the identifier
// and the packed value (the grid's centre a_j and the low B bits give u_j);
// each word is replaced by its identifier for the passes that follow.
template <int DB>
__global__ __launch_bounds__(kBlock) void unpack64_kernel(Batch b, uint64_t* __restrict__ words, int B,
                                                          int32_t* __restrict__ crd) {
    const int k = tile_instance(b, blockIdx.x);
    const Inst& I = b.inst[k];
    const int64_t lo = (int64_t)(blockIdx.x - I.tile0) * b.tile_pts;
    const int64_t hi = min(I.n, lo + b.tile_pts);
    const int W = b.D * B;
    const uint64_t low = (1ull << B) - 1ull;
    const int64_t half = (int64_t)1 << (B - 1);
    with_d<DB>(I.d, [&](auto dc) {
        constexpr int D = decltype(dc)::value;
        int sh[D];
        uint64_t fm[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            sh[j] = I.shift[j];
            fm[j] = I.bits[j] >= 64 ? ~0ull : ((1ull << I.bits[j]) - 1ull);
        }
        const double side = (double)I.eps / sqrt((double)D);
#pragma unroll 4
        for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
            const int64_t s = I.off + i;
            const uint64_t w = words[s];
            const uint64_t key = w >> W;
            int32_t y[DB];
#pragma unroll
            for (int j = 0; j < DB; ++j) y[j] = 0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const uint64_t g = (key >> sh[j]) & fm[j];
                const int64_t a = (int64_t)floor(((double)g + 0.5) * side);
                const uint64_t lb = (w >> (j * B)) & low;
                const uint64_t t = ((uint64_t)((int64_t)lb - a + half)) & low;
                y[j] = (int32_t)(a + (int64_t)t - half);
            }
            store_row<DB>(crd, s, y);
            words[s] = key;
        }
    });
}

hipError_t launch_unpack64(const Batch& b, uint64_t* words, int bits, int32_t* crd, hipStream_t st) {
    if (b.tiles == 0) return hipSuccess;
    GD_DISPATCH_D(b.D, (unpack64_kernel<D><<<dim3(b.tiles), dim3(kBlock), 0, st>>>(b, words, bits, crd)));
    return hipGetLastError();
}

template <int D>
struct FRow {
    float v[D];
};

// Sorted position s of instance k lies in [off_k, off_k + n_k): the same
// tiles as the input order.  Each thread keeps four rows in flight; a row of
// the input is fetched with one load of d floats.
template <int DB>
__global__ __launch_bounds__(kBlock) void gather_kernel(Batch b, const uint32_t* __restrict__ sidx,
                                                        int32_t* __restrict__ crd) {
    constexpr int U = 4;
    const int k = tile_instance(b, blockIdx.x);
    const Inst& I = b.inst[k];
    const int d = I.d;
    const int64_t lo = (int64_t)(blockIdx.x - I.tile0) * b.tile_pts;
    const int64_t hi = min(I.n, lo + b.tile_pts);
    int32_t mn[DB];
#pragma unroll
    for (int j = 0; j < DB; ++j) mn[j] = j < d ? I.mn[j] : 0;
    const float GD_GLOBAL* __restrict__ x = as_global(I.x);
    if (d == DB) {
        const FRow<DB> GD_GLOBAL* __restrict__ xr = reinterpret_cast<const FRow<DB> GD_GLOBAL*>(x);
        for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += U * kBlock) {
            uint32_t o[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = i0 + (int64_t)u * kBlock;
                // sidx of this range always lies in the instance; the clamp only guards the read
                o[u] = i < hi ? min((uint32_t)((int64_t)sidx[I.off + i] - I.off), (uint32_t)(I.n - 1)) : 0u;
            }
            FRow<DB> r[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (i0 + (int64_t)u * kBlock < hi) {
#pragma unroll
                    for (int j = 0; j < DB; ++j) r[u].v[j] = xr[o[u]].v[j];
                }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t i = i0 + (int64_t)u * kBlock;
                if (i < hi) {
                    int32_t y[DB];
#pragma unroll
                    for (int j = 0; j < DB; ++j) y[j] = (int)r[u].v[j] - mn[j];
                    store_row<DB>(crd, I.off + i, y);
                }
            }
        }
    } else {
        for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
            const int64_t s = I.off + i;
            const int64_t o = (int64_t)min((uint32_t)((int64_t)sidx[s] - I.off), (uint32_t)(I.n - 1));
            int32_t y[DB];
#pragma unroll
            for (int j = 0; j < DB; ++j) y[j] = j < d ? (int)x[o * d + j] - mn[j] : 0;
            store_row<DB>(crd, s, y);
        }
    }
}

hipError_t launch_gather(const Batch& b, const uint32_t* sidx, int32_t* crd, hipStream_t st) {
    if (b.tiles == 0) return hipSuccess;
    GD_DISPATCH_D(b.D, (gather_kernel<D><<<dim3(b.tiles), dim3(kBlock), 0, st>>>(b, sidx, crd)));
    return hipGetLastError();
}

template <typename K>
struct KeyChange {
    const K* k;
    // called for i < n only; both loads unconditional (no branch per element)
    __device__ uint32_t operator()(int64_t i) const {
        const K a = k[i];
        const K b = k[i > 0 ? i - 1 : 0];
        return (uint32_t)((i == 0) | (a != b));
    }
};

// Runs of equal identifiers, from the flag scan of "identifier changes
// here": the change at sorted position s starts grid c (its rank among the
// changes); end() closes the last run.
template <typename K>
struct CellWriter {
    Batch b;
    const K* skeys;
    uint32_t* cell_start;
    int32_t* ck;
    int64_t ck_stride;
    // s: first sorted position of grid c
    // Every load comes before the first store: a load issued after a store
    // would wait for it.
    __device__ void operator()(int64_t s, uint32_t c) const {
        const K key = skeys[s];
        int k = 0;
        if (b.count > 1) {
            const int ishift = b.hdr->inst_shift;
            k = (int)min(key_field(key, ishift, 64), (uint64_t)(b.count - 1));
            if (b.hdr->err & (kErrNotInteger | kErrKeyBits | kErrPlan)) k = (int)min(key_field(key, 0, 64), (uint64_t)(b.count - 1));
        }
        const Inst& I = b.inst[k];
        const int d = I.d;
        int32_t v[kMaxD];
#pragma unroll
        for (int j = 0; j < kMaxD; ++j) {
            v[j] = 0;
            if (j < b.D && j < d) v[j] = (int32_t)key_field(key, I.shift[j], I.bits[j]);
        }
        cell_start[c] = (uint32_t)s;
        ck[c] = k;
#pragma unroll
        for (int j = 0; j < kMaxD; ++j)
            if (j < b.D) ck[(int64_t)(j + 1) * ck_stride + c] = v[j];
    }
    __device__ void end(uint32_t ncell) const { cell_start[ncell] = (uint32_t)b.n; }
};

template <typename K>
hipError_t launch_cells(const Batch& b, const K* skeys, uint32_t* partial, uint32_t* cell_start,
                        int32_t* ck, int64_t ck_stride, hipStream_t st) {
    return scan_flags_apply(KeyChange<K>{skeys}, b.n, CellWriter<K>{b, skeys, cell_start, ck, ck_stride},
                            &b.hdr->ncell, partial, st);
}
template hipError_t launch_cells<uint32_t>(const Batch&, const uint32_t*, uint32_t*, uint32_t*, int32_t*,
                                           int64_t, hipStream_t);
template hipError_t launch_cells<uint64_t>(const Batch&, const uint64_t*, uint32_t*, uint32_t*, int32_t*,
                                           int64_t, hipStream_t);
template hipError_t launch_cells<Key128>(const Batch&, const Key128*, uint32_t*, uint32_t*, int32_t*, int64_t,
                                         hipStream_t);

// A grid starts a new node at level l iff it differs from the previous grid
// in one of the identifier rows 0..l (grids are in lexicographic order).
// Node-start flags of levels l0 .. l0 + nl - 1 for grid c, packed `bits`
// apart so one scan counts several levels: a grid starts a new node at level
// l iff it differs from the previous grid in one of the identifier rows
// 0..l (grids are in lexicographic order).
struct LevelFlags {
    const int32_t* ck;
    int64_t stride;
    const uint32_t* ncell;
    int l0, nl, bits;
    __device__ uint64_t operator()(int64_t c) const {
        if (c >= (int64_t)*ncell) return 0;
        bool diff = c == 0;
        uint64_t v = 0;
        for (int j = 0; j < l0 + nl; ++j) {
            if (!diff) diff = ck[(int64_t)j * stride + c] != ck[(int64_t)j * stride + c - 1];
            if (j >= l0 && diff) v |= 1ull << ((j - l0) * bits);
        }
        return v;
    }
};

// Unpacks the scan: per level, the nodes before grid c; at c = ncell that is
// the level's node count.
struct LevelExcl {
    uint32_t* excl[kMaxLevels];
    uint32_t* count;
    const uint32_t* ncell;
    int l0, nl, bits, levels;
    __device__ void operator()(int64_t c, uint64_t ex, uint64_t) const {
        const uint64_t mask = (1ull << bits) - 1ull;
        const bool last = c == (int64_t)*ncell;
        for (int k = 0; k < nl; ++k) {
            const uint32_t v = (uint32_t)((ex >> (k * bits)) & mask);
            excl[k][c] = v;
            if (last) count[l0 + k] = v;
        }
        if (last && l0 == 0) count[levels - 1] = (uint32_t)c;  // the last level's nodes are the grids
    }
};

struct TreeBuild {
    int32_t* key[kMaxLevels];
    uint32_t* child[kMaxLevels];
    const uint32_t* excl[kMaxLevels];  // per level: nodes before grid c (c in [0, ncell])
};

__global__ __launch_bounds__(kBlock) void tree_kernel(const int32_t* __restrict__ ck, int64_t stride,
                                                      const uint32_t* ncell_dev, int levels, TreeBuild tb) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t ncell = *ncell_dev;
    if (c > ncell) return;
    for (int l = 0; l + 1 < levels; ++l) {
        if (c == ncell || tb.excl[l][c + 1] != tb.excl[l][c]) {
            const uint32_t a = tb.excl[l][c];
            if (c < ncell) tb.key[l][a] = ck[(int64_t)l * stride + c];
            // children: the level-(l+1) node that starts at grid c; the last level's nodes are the grids
            tb.child[l][a] = (l + 2 < levels) ? tb.excl[l + 1][c] : (uint32_t)c;
        }
    }
}

hipError_t launch_tree(const GridView& g, uint32_t* level_excl, uint32_t* partial, int32_t* const* tkey,
                       uint32_t* const* tchild, hipStream_t st) {
    const int levels = g.D + 1;
    uint32_t* level_count = g.b.hdr->level_count;
    TreeBuild tb{};
    for (int l = 0; l + 1 < levels; ++l) {
        tb.key[l] = tkey[l];
        tb.child[l] = tchild[l];
        tb.excl[l] = level_excl + (int64_t)l * (g.ncell + 1);
    }
    // several levels per scan: counts are at most ncell + 1
    int bits = 1;
    while (((uint64_t)g.ncell + 1) >> bits) ++bits;
    const int per = 64 / bits;
    for (int l0 = 0; l0 + 1 < levels; l0 += per) {
        const int nl = std::min(per, levels - 1 - l0);
        LevelExcl out{};
        for (int k = 0; k < nl; ++k) out.excl[k] = level_excl + (int64_t)(l0 + k) * (g.ncell + 1);
        out.count = level_count;
        out.ncell = g.ncell_dev;
        out.l0 = l0;
        out.nl = nl;
        out.bits = bits;
        out.levels = levels;
        hipError_t e = scan_apply<uint64_t>(LevelFlags{g.ck, g.ck_stride, g.ncell_dev, l0, nl, bits}, g.ncell + 1,
                                            out, (uint64_t*)nullptr, reinterpret_cast<uint64_t*>(partial), st);
        if (e != hipSuccess) return e;
    }
    if (g.ncell == 0) return hipGetLastError();
    tree_kernel<<<dim3(grid_for(g.ncell + 1)), dim3(kBlock), 0, st>>>(g.ck, g.ck_stride, g.ncell_dev, levels, tb);
    return hipGetLastError();
}

}  // namespace gd
