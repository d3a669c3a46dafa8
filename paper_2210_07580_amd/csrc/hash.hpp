// Open-addressing hash tables keyed by packed grid identifiers, shared by
// the output pass (identifier -> cluster label) and the direct-hashing
// neighbour query (identifier -> grid index).  The all-ones identifier marks
// an empty slot.
#pragma once

#include "common.hpp"

namespace gd {

template <typename K>
struct HashSlot;
template <>
struct alignas(8) HashSlot<uint32_t> {
    uint32_t key;
    int32_t val;
};
template <>
struct alignas(16) HashSlot<uint64_t> {
    uint64_t key;
    int32_t val;
    int32_t pad;
};

// Buckets of 16 bytes (2 slots of u32 identifiers, 1 of u64) at load <= 1/4
// (<= 1/8 up to 2^20 grids): a lookup reads one bucket with a single 16-byte
// load and almost always ends there.  The table is hit at random addresses,
// one per lane, so the cost of a lookup is set by the cache lines each load
// instruction touches, not by the bytes: one load per lookup rather than a
// wider bucket.
template <typename K>
constexpr int kBucketSlots = 16 / (int)sizeof(HashSlot<K>);
template <typename K>
constexpr int kBucketShift = sizeof(K) == 4 ? 1 : 0;

template <typename K>
__device__ __forceinline__ uint64_t hash_bucket(K key, int bbits) {
    return ((uint64_t)key * 0x9E3779B97F4A7C15ull) >> (64 - bbits);
}

__device__ __forceinline__ uint32_t cas_key(uint32_t* p, uint32_t cmp, uint32_t v) { return atomicCAS(p, cmp, v); }
__device__ __forceinline__ uint64_t cas_key(uint64_t* p, uint64_t cmp, uint64_t v) {
    return (uint64_t)atomicCAS(reinterpret_cast<unsigned long long*>(p), (unsigned long long)cmp,
                               (unsigned long long)v);
}

// Look `key` up in one loaded bucket: 1 found (val set), 0 absent (the
// bucket has an empty slot: slots fill in order and are never freed), -1
// look in the next bucket.
__device__ __forceinline__ int bucket_match(const uint4& q, uint32_t key, int32_t& val) {
    if (q.x == key) {
        val = (int32_t)q.y;
        return 1;
    }
    if (q.z == key) {
        val = (int32_t)q.w;
        return 1;
    }
    return (q.x == ~0u || q.z == ~0u) ? 0 : -1;
}
__device__ __forceinline__ int bucket_match(const uint4& q, uint64_t key, int32_t& val) {
    const uint64_t k = (uint64_t)q.x | ((uint64_t)q.y << 32);
    if (k == key) {
        val = (int32_t)q.z;
        return 1;
    }
    return k == ~0ull ? 0 : -1;
}

template <typename K>
__device__ __forceinline__ uint4 load_bucket(const HashSlot<K>* tab, uint64_t b) {
    return *reinterpret_cast<const uint4*>(tab + (b << kBucketShift<K>));
}

// Tables hold 2^bits slots plus one: the all-ones identifier marks an empty
// slot, so a grid with that identifier keeps its value in the extra slot at
// index 2^bits.  Clearing writes the empty key and `empty_val` everywhere.
template <typename K>
__global__ __launch_bounds__(kBlock) void hash_clear_kernel(HashSlot<K>* tab, int64_t slots, int32_t empty_val) {
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < slots; i += (int64_t)gridDim.x * kBlock) {
        tab[i].key = ~K(0);
        tab[i].val = empty_val;
    }
}

// Value of `key` in a table filled by grid_table_insert, or the extra slot's
// value for the all-ones key; a missing key returns -1 (the probe stops at
// the first bucket with an empty slot: slots fill in order and are never
// freed).
template <typename K>
__device__ __forceinline__ int32_t grid_table_find(const HashSlot<K>* __restrict__ tab, int bits, K key) {
    if (key == ~K(0)) return tab[1ull << bits].val;
    const int bbits = bits - kBucketShift<K>;
    const uint64_t bmask = (1ull << bbits) - 1ull;
    uint64_t b = hash_bucket(key, bbits);
    for (uint64_t probes = 0; probes <= bmask; ++probes, b = (b + 1) & bmask) {
        int32_t val;
        const int r = bucket_match(load_bucket(tab, b), key, val);
        if (r >= 0) return r ? val : -1;
    }
    return -1;
}

// Insert (key, val); the table's load stays below one half, so a free slot
// is always found.
template <typename K>
__device__ __forceinline__ void grid_table_insert(HashSlot<K>* tab, int bits, K key, int32_t val) {
    if (key == ~K(0)) {
        tab[1ull << bits].val = val;
        return;
    }
    const int bbits = bits - kBucketShift<K>;
    const uint64_t bmask = (1ull << bbits) - 1ull;
    for (uint64_t b = hash_bucket(key, bbits);; b = (b + 1) & bmask) {
        HashSlot<K>* bucket = tab + (b << kBucketShift<K>);
        for (int j = 0; j < kBucketSlots<K>; ++j) {
            if (cas_key(&bucket[j].key, ~K(0), key) == ~K(0)) {
                bucket[j].val = val;
                return;
            }
        }
    }
}

}  // namespace gd
