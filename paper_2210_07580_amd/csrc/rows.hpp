// The last pass of the identifier sort (Algorithm 1) of a single instance
// with packed rows (launch.hpp, pack_fits): instead of the sorted packed
// values, it writes each point's sorted row, its index and its identifier,
// so that no separate pass reads the sorted values back.  Each row is
// rebuilt as unpack_kernel rebuilds it: the grid's centre a_j (from the
// identifier) and the low B = pack_bits(D) bits of u_j = x_j - mn_j (from the
// value) leave exactly one candidate for u_j within 2^(B-1) of a_j.
#pragma once

#include "common.hpp"

namespace gd {

template <int D>
struct PackedRowsOut {
    const Inst* inst;  // device: the instance (its identifier layout)
    int32_t* crd;      // sorted rows (row_stride(D) words each)
    uint32_t* keys;    // sorted identifiers (bound to the pass's key buffer)
    uint32_t* sidx;    // sorted index (bound to the pass's value buffer)
    int sh[D];
    uint32_t fm[D];
    double side;

    void bind(uint32_t* k, uint64_t* v) {
        keys = k;
        sidx = reinterpret_cast<uint32_t*>(v);
    }
    __device__ void begin() {
        const Inst& I = inst[0];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            sh[j] = I.shift[j];
            fm[j] = I.bits[j] >= 32 ? 0xFFFFFFFFu : ((1u << I.bits[j]) - 1u);
        }
        side = (double)I.eps / sqrt((double)D);
    }
    __device__ void store(uint32_t pos, uint32_t key, uint64_t v) const {
        constexpr int B = pack_bits(D);
        constexpr uint64_t kLow = B >= 32 ? 0xFFFFFFFFull : ((1ull << B) - 1ull);
        constexpr int64_t kHalf = (int64_t)1 << (B - 1);
        const uint64_t packed = v >> 32;
        int32_t y[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const uint32_t g = (key >> sh[j]) & fm[j];
            const int64_t a = (int64_t)floor(((double)g + 0.5) * side);
            const uint64_t low = (packed >> (j * B)) & kLow;
            const uint64_t t = ((uint64_t)((int64_t)low - a + kHalf)) & kLow;
            y[j] = (int32_t)(a + (int64_t)t - kHalf);
        }
        store_row<D>(crd, pos, y);
        keys[pos] = key;
        sidx[pos] = (uint32_t)v;
    }
};

}  // namespace gd
