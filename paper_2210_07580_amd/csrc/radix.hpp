// Stable LSD radix sort of (key, value) pairs (u32 or u64 values) for the
// grid identifiers of Section 4.1 (Algorithm 1 orders the points by
// identifier with a radix sort).  A sort of B bits takes ceil(B / 8) passes
// of equal digits of at most 8 bits (wider digits cost more per pass than
// the pass they save: a 4x larger offset table to scan, more ranking
// ballots and less occupancy).
//
// Each pass is reduce-then-scan: (1) every workgroup builds the digit
// histogram of its tile (4096 keys; 2048 with 64-bit values; 1024 in sorts
// of at most 2^21 keys) in LDS (one sub-histogram per wave to cut atomic
// contention); (2) a device-wide exclusive scan over the digit-major
// [bins][tiles] table gives every (digit, tile) its output base; (3) every
// workgroup re-reads its tile; each wave takes a run of a quarter of it
// (consecutive keys) and ranks them among equal digits with wave64 ballots
// (one ballot per digit bit gives the lanes holding the same digit; the rank
// is the popcount below the lane plus the wave's running count of that
// digit, kept in LDS), one scan over (digit, wave) turns the counts into
// local slots, the keys are placed in LDS in digit order and written out run
// by run, so that neighbouring lanes store to neighbouring addresses.  Ranks
// follow input order, so every pass is stable.
#pragma once

#include <algorithm>

#include "scan.hpp"

namespace gd {

// Keys per thread of a tile: 16 (4096-key tiles), or 4 (1024-key tiles) for
// sorts of at most kRadixSmallMax keys, which would otherwise have fewer
// tiles than the GPU has compute units, each ranked by one long chain of
// wave steps.  Sorts with 64-bit values take 8 (2048-key tiles): a 4096-key
// tile of them would stage 48 KB of keys and values in LDS and leave room
// for two workgroups per compute unit.
constexpr int kRadixItemsBig = 16;
constexpr int kRadixItemsWide = 8;
constexpr int kRadixItemsSmall = 4;
constexpr int64_t kRadixSmallMax = 1 << 21;

template <typename K>
constexpr int radix_max_bits() { return 8; }
template <typename K>
constexpr int radix_max_bins() { return 1 << radix_max_bits<K>(); }

// Two-word identifiers take the 2048-key tiles too (a 4096-key tile of them
// with their values would not fit the LDS).
inline int radix_items(int64_t n, int value_bytes = 4, int key_bytes = 4) {
    return n <= kRadixSmallMax ? kRadixItemsSmall
                               : (value_bytes > 4 || key_bytes > 8) ? kRadixItemsWide : kRadixItemsBig;
}
inline int64_t radix_tiles(int64_t n, int value_bytes = 4) {
    const int64_t tile = (int64_t)kBlock * radix_items(n, value_bytes);
    return (n + tile - 1) / tile;
}
inline int64_t radix_scratch_words_for(int64_t n, int value_bytes) {
    const int64_t t = radix_tiles(n, value_bytes);
    constexpr int64_t bins = 1 << 8;
    return 2 * bins * t + scan_partial_cap(bins * t) + 4;
}
// u32 entries of scratch enough for a sort of any m <= n keys (any key and
// value type)
inline int64_t radix_scratch_words(int64_t n) {
    const int64_t small = std::min(n, kRadixSmallMax);
    return std::max(std::max(radix_scratch_words_for(n, 4), radix_scratch_words_for(n, 8)),
                    radix_scratch_words_for(small, 4));
}

// Neighbouring tiles write neighbouring addresses (their counts in the
// digit-major histogram table, their runs of one digit in the scatter), so
// workgroup b takes tile xcd_order(b): every XCD then writes one contiguous
// range, and a line is written from one L2 instead of being merged from
// partial copies in several.
template <typename K, int kItems>
__global__ __launch_bounds__(kBlock) void radix_hist_kernel(const K* __restrict__ keys, int64_t n, int shift, int rbits,
                                                            uint32_t* __restrict__ hist, int64_t tiles) {
    constexpr int kMaxBins = radix_max_bins<K>();
    __shared__ uint32_t h[kWavesPerBlock][kMaxBins];
    const int bins = 1 << rbits;
    for (int i = threadIdx.x; i < kWavesPerBlock * kMaxBins; i += kBlock) (&h[0][0])[i] = 0;
    __syncthreads();
    constexpr int kTile = kBlock * kItems;
    const int64_t tile = xcd_order(blockIdx.x, tiles);
    const int64_t base = tile * kTile;
    const int w = wave_id();
    const uint32_t mask = (uint32_t)bins - 1u;
    // all loads of the tile in flight before the first count
    K k[kItems];
    const bool full = base + kTile <= n;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
        k[r] = (full || i < n) ? keys[i] : K(0);
    }
    // Lanes hold neighbouring keys, and after the first passes a run of
    // neighbouring keys often shares the digit (a whole grid's points do in
    // the last pass); same-address LDS atomics of one instruction serialise.
    // So the keys that share the digit of the first lane still to count are
    // counted by one atomic, as long as such groups have eight keys or more
    // (at most eight groups); the rest count one by one (on random digits:
    // one check per round).
    const int lane = lane_id();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t i = base + (int64_t)r * kBlock + threadIdx.x;
        const bool v = full || i < n;
        const uint32_t dg = (uint32_t)(k[r] >> shift) & mask;
        uint64_t rem = ballot(v);
        while (rem) {
            const int l0 = ffs64(rem);
            const uint32_t d0 = readlane(dg, l0);
            const uint64_t m = ballot(dg == d0) & rem;
            const uint32_t c = (uint32_t)popc64(m);
            if (c < 8u) break;
            if (lane == l0) atomicAdd(&h[w][d0], c);
            rem &= ~m;
        }
        if ((rem >> lane) & 1ull) atomicAdd(&h[w][dg], 1u);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < bins; t += kBlock) {
        uint32_t s = 0;
#pragma unroll
        for (int ww = 0; ww < kWavesPerBlock; ++ww) s += h[ww][t];
        hist[(int64_t)t * tiles + tile] = s;
    }
}

// Where a scatter pass puts each (key, value) at its sorted slot: the next
// pass's buffers, or (PackedRowsOut, the last pass of the identifier sort)
// something derived from them.
template <typename K, typename V>
struct PairOut {
    K* keys;
    V* vals;
    void bind(K* k, V* v) {
        keys = k;
        vals = v;
    }
    __device__ void begin() {}
    __device__ void store(uint32_t pos, const K& k, const V& v) const {
        keys[pos] = k;
        vals[pos] = v;
    }
};

template <typename K, typename V, bool kIota, int kItems, typename Out>
__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(const K* __restrict__ keys, const V* __restrict__ vals,
                                                               Out out, int64_t n, int shift, int rbits,
                                                               const uint32_t* __restrict__ offs, int64_t tiles) {
    constexpr int kMaxBins = radix_max_bins<K>();
    constexpr int kDigitsPerThread = kMaxBins / kBlock;  // 4 or 2
    constexpr int kTile = kBlock * kItems;
    constexpr int kPerWave = kTile / kWavesPerBlock;       // 64 kItems consecutive keys per wave
    constexpr int kIters = kPerWave / kWave;               // kItems
    __shared__ K skey[kTile];                               // the tile, ordered by digit (stable)
    __shared__ V sval[kTile];
    __shared__ uint32_t wcnt[kWavesPerBlock][kMaxBins];     // keys per (wave, digit), then first local slot
    __shared__ uint32_t gbase[kMaxBins];                    // global slot of a digit's first key, minus its local start
    __shared__ uint32_t wsum[kWavesPerBlock];
    const int t = threadIdx.x;
    const int w = wave_id();
    const int lane = lane_id();
    const int bins = 1 << rbits;
    const uint32_t mask = (uint32_t)bins - 1u;
    for (int i = t; i < kWavesPerBlock * kMaxBins; i += kBlock) (&wcnt[0][0])[i] = 0;
    __syncthreads();
    // neighbouring tiles on one XCD (see xcd_order): their runs of a digit are
    // neighbours in the output
    const int64_t tile = xcd_order(blockIdx.x, tiles);
    const int64_t base = tile * kTile;
    const int tile_n = (int)min((int64_t)kTile, n - base);
    const uint64_t lt = lanemask_lt();
    // 1. each wave ranks its own run of keys among equal digits, in order,
    //    with wave-private counters (no workgroup barrier)
    K k[kIters];
    V v[kIters];
    uint32_t dr[kIters];  // digit << 16 | rank within the wave
#pragma unroll
    for (int it = 0; it < kIters; ++it) {
        const int li = w * kPerWave + it * kWave + lane;
        const bool valid = li < tile_n;
        k[it] = valid ? keys[base + li] : K(0);
        v[it] = valid ? (kIota ? (V)(base + li) : vals[base + li]) : V(0);
    }
#pragma unroll
    for (int it = 0; it < kIters; ++it) {
        const int li = w * kPerWave + it * kWave + lane;
        const bool valid = li < tile_n;
        const uint32_t dg = (uint32_t)(k[it] >> shift) & mask;
        // lanes with the same digit: one ballot per digit bit; the digit bits
        // above rbits are 0 in every lane and leave the mask unchanged.  The
        // halves are kept as 32-bit words and combined as p & ~(m ^ x), which
        // gfx950 evaluates with three-input bit operations.
        const uint64_t vm = ballot(valid);
        uint32_t plo = (uint32_t)vm, phi = (uint32_t)(vm >> 32);
#pragma unroll
        for (int b = 0; b < radix_max_bits<K>(); ++b) {
            const uint32_t x = (uint32_t)(((int32_t)(dg << (31 - b))) >> 31);  // all ones where bit b is set
            const uint64_t m = ballot(x != 0u);
            plo &= ~((uint32_t)m ^ x);
            phi &= ~((uint32_t)(m >> 32) ^ x);
        }
        const uint64_t peers = ((uint64_t)phi << 32) | plo;
        const uint32_t before = valid ? wcnt[w][dg] : 0u;
        wave_sync();
        const uint32_t rank = before + (uint32_t)popc64(peers & lt);
        if (valid && (peers & lt) == 0) wcnt[w][dg] = before + (uint32_t)popc64(peers);
        wave_sync();
        dr[it] = (dg << 16) | rank;
    }
    __syncthreads();
    // 2. local start of each (wave, digit): digits in order, waves in order;
    //    thread t owns digits [t * kDigitsPerThread, +kDigitsPerThread)
    {
        uint32_t c[kDigitsPerThread][kWavesPerBlock], tot[kDigitsPerThread], mine = 0;
#pragma unroll
        for (int q = 0; q < kDigitsPerThread; ++q) {
            const int dg = t * kDigitsPerThread + q;
            tot[q] = 0;
#pragma unroll
            for (int ww = 0; ww < kWavesPerBlock; ++ww) {
                c[q][ww] = dg < bins ? wcnt[ww][dg] : 0u;
                tot[q] += c[q][ww];
            }
            mine += tot[q];
        }
        uint32_t all;
        uint32_t acc = block_excl_scan(mine, wsum, all);
#pragma unroll
        for (int q = 0; q < kDigitsPerThread; ++q) {
            const int dg = t * kDigitsPerThread + q;
            if (dg < bins) {
                gbase[dg] = offs[(int64_t)dg * tiles + tile] - acc;
#pragma unroll
                for (int ww = 0; ww < kWavesPerBlock; ++ww) {
                    wcnt[ww][dg] = acc;
                    acc += c[q][ww];
                }
            }
        }
    }
    __syncthreads();
    // 3. place the keys in LDS in digit order
#pragma unroll
    for (int it = 0; it < kIters; ++it) {
        const int li = w * kPerWave + it * kWave + lane;
        if (li < tile_n) {
            const uint32_t pos = wcnt[w][dr[it] >> 16] + (dr[it] & 0xFFFFu);
            skey[pos] = k[it];
            sval[pos] = v[it];
        }
    }
    __syncthreads();
    // 4. write the digit runs out in order: consecutive threads, consecutive slots
    out.begin();
    for (int j = t; j < tile_n; j += kBlock) {
        const K kk = skey[j];
        const uint32_t dg = (uint32_t)(kk >> shift) & mask;
        const uint32_t pos = gbase[dg] + (uint32_t)j;
        out.store(pos, kk, sval[j]);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void iota_kernel(T* v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) v[i] = (T)i;
}

template <typename K, typename V = uint32_t>
struct RadixResult {
    K* keys;
    V* vals;
    bool last_fused;  // the last pass wrote through `last` (false: no pass ran, or none was given)
};

// Sorts keys[0..n) (and vals) on their bits [lo, lo + bits).  keys/vals and
// keys_alt/vals_alt are ping-pong buffers; the result lands in one of them.
// With keys_spare, the passes after the first alternate between keys_alt
// and keys_spare, so keys[] keeps the input order.
// If vals_iota, vals[] is not read and the values start as 0..n-1.
// `scratch` needs radix_scratch_words(n) u32.  With `last`, the last pass
// stores through a copy of it, bound to that pass's output buffers.
template <typename K, typename V = uint32_t, typename Last = PairOut<K, V>>
hipError_t radix_sort_pairs(K* keys, V* vals, K* keys_alt, V* vals_alt, int64_t n, int bits,
                            bool vals_iota, uint32_t* scratch, hipStream_t st, RadixResult<K, V>* out,
                            K* keys_spare = nullptr, int lo = 0, const Last* last = nullptr) {
    K* kin = keys;
    V* vin = vals;
    K* kout = keys_alt;
    V* vout = vals_alt;
    bool first = true;
    const int items = radix_items(n, (int)sizeof(V), (int)sizeof(K));
    const int64_t tiles = (n + (int64_t)kBlock * items - 1) / ((int64_t)kBlock * items);
    uint32_t* hist = scratch;
    uint32_t* offs = scratch + (int64_t)radix_max_bins<uint32_t>() * tiles;
    uint32_t* partial = offs + (int64_t)radix_max_bins<uint32_t>() * tiles;
    bool iota = vals_iota;
    bool fused = false;
    const int passes = bits <= 0 ? 0 : (bits + radix_max_bits<K>() - 1) / radix_max_bits<K>();
    const int rbits = passes ? (bits + passes - 1) / passes : 0;
    for (int p = 0, shift = lo; p < passes; ++p, shift += rbits) {
        if (n == 0) break;
        const int64_t bins = (int64_t)1 << rbits;
        const dim3 grid((unsigned)tiles), block(kBlock);
        if (items == kRadixItemsSmall)
            radix_hist_kernel<K, kRadixItemsSmall><<<grid, block, 0, st>>>(kin, n, shift, rbits, hist, tiles);
        else if (items == kRadixItemsWide)
            radix_hist_kernel<K, kRadixItemsWide><<<grid, block, 0, st>>>(kin, n, shift, rbits, hist, tiles);
        else
            radix_hist_kernel<K, kRadixItemsBig><<<grid, block, 0, st>>>(kin, n, shift, rbits, hist, tiles);
        hipError_t e = scan_exclusive<uint32_t>(ArrayInput<uint32_t>{hist}, bins * tiles, offs, (uint32_t*)nullptr,
                                                partial, st);
        if (e != hipSuccess) return e;
        auto scatter = [&](auto o) {
            using O = decltype(o);
            if (items == kRadixItemsSmall) {
                if (iota)
                    radix_scatter_kernel<K, V, true, kRadixItemsSmall, O><<<grid, block, 0, st>>>(
                        kin, vin, o, n, shift, rbits, offs, tiles);
                else
                    radix_scatter_kernel<K, V, false, kRadixItemsSmall, O><<<grid, block, 0, st>>>(
                        kin, vin, o, n, shift, rbits, offs, tiles);
            } else if (items == kRadixItemsWide) {
                if (iota)
                    radix_scatter_kernel<K, V, true, kRadixItemsWide, O><<<grid, block, 0, st>>>(
                        kin, vin, o, n, shift, rbits, offs, tiles);
                else
                    radix_scatter_kernel<K, V, false, kRadixItemsWide, O><<<grid, block, 0, st>>>(
                        kin, vin, o, n, shift, rbits, offs, tiles);
            } else {
                if (iota)
                    radix_scatter_kernel<K, V, true, kRadixItemsBig, O><<<grid, block, 0, st>>>(
                        kin, vin, o, n, shift, rbits, offs, tiles);
                else
                    radix_scatter_kernel<K, V, false, kRadixItemsBig, O><<<grid, block, 0, st>>>(
                        kin, vin, o, n, shift, rbits, offs, tiles);
            }
        };
        if (last && p == passes - 1) {
            Last o = *last;
            o.bind(kout, vout);
            scatter(o);
            fused = true;
        } else {
            PairOut<K, V> o;
            o.bind(kout, vout);
            scatter(o);
        }
        iota = false;
        K* tk = kin; kin = kout; kout = (first && keys_spare) ? keys_spare : tk;
        first = false;
        V* tv = vin; vin = vout; vout = tv;
    }
    if (iota && n > 0) {  // no pass ran: the values must still be 0..n-1
        iota_kernel<V><<<dim3(grid_for(n)), dim3(kBlock), 0, st>>>(vin, n);
    }
    out->keys = kin;
    out->vals = vin;
    out->last_fused = fused;
    return hipGetLastError();
}

}  // namespace gd
