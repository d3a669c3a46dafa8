// Learned proposal for the merge step: per-grid summaries, pair features
// and the 16 -> 64 -> 64 -> 2 scorer, shared by the merge kernel, the
// harvesting kernel and the training kernel.
//
// The scorer is this project's addition.  Output 0 is the logit that the
// pair of core grids merges (used to test likely merges first), output 1
// the logit that FastMerging costs fewer distance evaluations when it
// starts from the second grid.  FastMerging still decides every pair
// exactly (Theorem 2); a proposal only changes the order of the tests, the
// starting side, and the starting point (the core point of the starting
// grid that lies furthest towards the other grid along their dominant axis,
// instead of the paper's random point).
#pragma once

#include <hip/hip_fp16.h>

#include "common.hpp"
#include "launch.hpp"

namespace gd {

constexpr int kFeat = 16, kHid = 64, kOut = 2;
constexpr int oW1 = 0;
constexpr int oB1 = oW1 + kHid * kFeat;  // 1024
constexpr int oW2 = oB1 + kHid;          // 1088
constexpr int oB2 = oW2 + kHid * kHid;   // 5184
constexpr int oW3 = oB2 + kHid;          // 5248
constexpr int oB3 = oW3 + kOut * kHid;   // 5376
constexpr int kParams = oB3 + kOut;      // 5378
constexpr float kLambda = 0.5f;          // weight of the side loss

struct TrainArgs {
    const __half* x;        // S x 16 features
    const float* t;         // S x 3 targets (y0, y1, w1)
    const uint32_t* order;  // steps x batch sample indices
    int steps, batch;
    float lr;
    int adam_t0;            // Adam steps already taken
    float* params;          // 5378 FP32 master weights (in/out)
    float* m;               // Adam moments (in/out)
    float* v;
    float* loss;            // steps (mean loss of each step's batch), or null
    float* grad;            // 5378: gradient of the first step's batch, or null
    int update;             // 0: compute only
    __half* blob;           // 5378 FP16 weights after training, or null
};

// Summary of one core grid's core points.
struct CellSummary {
    float cen[kMaxD];         // centroid
    int32_t lo[kMaxD];        // bounding box
    int32_t hi[kMaxD];
    uint32_t rep[2 * kMaxD];  // rep[2k] / rep[2k+1]: position of the smallest / largest coordinate k
};

// The scorer's weights as a workgroup keeps them in LDS (FP16 values
// widened to FP32; W1 and W2 transposed so lane u reads column u).
struct MlpLds {
    float w1t[kFeat][kHid];
    float w2t[kHid][kHid + 1];
    float b1[kHid], b2[kHid];
    float w3[kOut][kHid];
    float b3[kOut];
};

// Load the FP16 parameter vector (layout: W1 [64x16], b1, W2 [64x64], b2,
// W3 [2x64], b3) into LDS.  All threads of the workgroup call it.
__device__ inline void mlp_load(MlpLds& m, const __half* __restrict__ p) {
    for (int i = threadIdx.x; i < kHid * kFeat; i += blockDim.x) {
        const int u = i / kFeat, k = i % kFeat;
        m.w1t[k][u] = __half2float(p[oW1 + i]);
    }
    for (int i = threadIdx.x; i < kHid * kHid; i += blockDim.x) {
        const int u = i / kHid, k = i % kHid;
        m.w2t[k][u] = __half2float(p[oW2 + i]);
    }
    for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
        m.b1[i] = __half2float(p[oB1 + i]);
        m.b2[i] = __half2float(p[oB2 + i]);
        m.w3[0][i] = __half2float(p[oW3 + i]);
        m.w3[1][i] = __half2float(p[oW3 + kHid + i]);
    }
    if (threadIdx.x < kOut) m.b3[threadIdx.x] = __half2float(p[oB3 + threadIdx.x]);
}

// The scorer on the matrix cores: 16 pairs at a time as three small GEMMs
// with v_mfma_f32_16x16x16_f16 (FP16 operands, FP32 accumulation), the same
// arithmetic as mlp_forward_wave (hidden activations rounded to FP16).
// Operand layout of the 16x16x16 instruction, lane l = 0..63, element j:
//   A (rows x k):  A[l % 16][4 (l / 16) + j]
//   B (k x cols):  B[4 (l / 16) + j][l % 16]
//   D (rows x cols): D[4 (l / 16) + j][l % 16]
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

struct MlpMfma {
    _Float16 w1[kHid][kFeat];  // W1 as stored: row = hidden unit, column = feature
    _Float16 w2[kHid][kHid];   // W2: row = output unit, column = input unit
    float b1[kHid], b2[kHid];
    float w3[kOut][kHid];
    float b3[kOut];
};

__device__ inline void mlp_mfma_load(MlpMfma& m, const __half* __restrict__ p) {
    for (int i = threadIdx.x; i < kHid * kFeat; i += blockDim.x)
        (&m.w1[0][0])[i] = (_Float16)__half2float(p[oW1 + i]);
    for (int i = threadIdx.x; i < kHid * kHid; i += blockDim.x)
        (&m.w2[0][0])[i] = (_Float16)__half2float(p[oW2 + i]);
    for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
        m.b1[i] = __half2float(p[oB1 + i]);
        m.b2[i] = __half2float(p[oB2 + i]);
        m.w3[0][i] = __half2float(p[oW3 + i]);
        m.w3[1][i] = __half2float(p[oW3 + kHid + i]);
    }
    if (threadIdx.x < kOut) m.b3[threadIdx.x] = __half2float(p[oB3 + threadIdx.x]);
}

// Scratch of one wave: the 16 feature rows and the first hidden layer.
struct MlpMfmaScratch {
    _Float16 feat[16][kFeat];
    _Float16 h1[16][kHid];
};

// Scores of the 16 feature rows in s.feat (all lanes call it).  On return
// lane l holds z[o][r] for rows r = 4 (l / 16) + j in z0[j], z1[j].
__device__ inline void mlp_forward_mfma(const MlpMfma& m, MlpMfmaScratch& s, float (&z0)[4], float (&z1)[4]) {
    const int l = lane_id();
    const int r = l & 15, g = l >> 4;
    const float4_t zero = {0.f, 0.f, 0.f, 0.f};
    // layer 1: [16 x 16] . [16 x 64]
    const half4_t a1 = *reinterpret_cast<const half4_t*>(&s.feat[r][4 * g]);
#pragma unroll
    for (int nb = 0; nb < kHid / 16; ++nb) {
        const half4_t b = *reinterpret_cast<const half4_t*>(&m.w1[nb * 16 + r][4 * g]);
        const float4_t d = __builtin_amdgcn_mfma_f32_16x16x16f16(a1, b, zero, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) s.h1[4 * g + j][nb * 16 + r] = (_Float16)fmaxf(d[j] + m.b1[nb * 16 + r], 0.f);
    }
    wave_sync();
    // layer 2: [16 x 64] . [64 x 64], then layer 3 on the result
    float p0[4] = {0.f, 0.f, 0.f, 0.f}, p1[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int nb = 0; nb < kHid / 16; ++nb) {
        float4_t acc = zero;
#pragma unroll
        for (int kb = 0; kb < kHid / 16; ++kb) {
            const half4_t a = *reinterpret_cast<const half4_t*>(&s.h1[r][kb * 16 + 4 * g]);
            const half4_t b = *reinterpret_cast<const half4_t*>(&m.w2[nb * 16 + r][kb * 16 + 4 * g]);
            acc = __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, acc, 0, 0, 0);
        }
        const int col = nb * 16 + r;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float h2 = (float)(_Float16)fmaxf(acc[j] + m.b2[col], 0.f);
            p0[j] += m.w3[0][col] * h2;
            p1[j] += m.w3[1][col] * h2;
        }
    }
    // sum over the 16 columns each lane group holds
#pragma unroll
    for (int j = 0; j < 4; ++j) {
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            p0[j] += __shfl_xor(p0[j], o);
            p1[j] += __shfl_xor(p1[j], o);
        }
        z0[j] = p0[j] + m.b3[0];
        z1[j] = p1[j] + m.b3[1];
    }
    wave_sync();  // s.h1 may be rewritten by the next call
}

// Forward pass for one pair on a whole wave: lane u owns hidden unit u.
// `f` is uniform across the wave (the features already rounded to FP16);
// `hbuf` is 64 floats of the wave's own LDS.  Hidden activations are
// rounded to FP16 like the stored inputs; sums accumulate in FP32.
struct MlpTrace {
    float a1, h1, a2, h2;  // this lane's unit
    float z0, z1;          // uniform
};

__device__ inline MlpTrace mlp_forward_wave(const MlpLds& m, const float (&f)[kFeat], float* hbuf) {
    const int u = lane_id();
    MlpTrace r;
    float a = m.b1[u];
#pragma unroll
    for (int k = 0; k < kFeat; ++k) a += m.w1t[k][u] * f[k];
    r.a1 = a;
    r.h1 = __half2float(__float2half(fmaxf(a, 0.f)));
    hbuf[u] = r.h1;
    wave_sync();
    float a2 = m.b2[u];
#pragma unroll 8
    for (int k = 0; k < kHid; ++k) a2 += m.w2t[k][u] * hbuf[k];
    r.a2 = a2;
    r.h2 = __half2float(__float2half(fmaxf(a2, 0.f)));
    r.z0 = wave_sum(m.w3[0][u] * r.h2) + m.b3[0];
    r.z1 = wave_sum(m.w3[1][u] * r.h2) + m.b3[1];
    wave_sync();  // hbuf may be rewritten by the caller's next pair
    return r;
}

// Position (within grid a's core set) of a's core point furthest towards
// grid b along the dominant axis of b's centroid minus a's.
__device__ inline uint32_t rep_towards(const CellSummary& a, const CellSummary& b, int d) {
    int best = 0;
    float bv = -1.f, bs = 0.f;
    for (int k = 0; k < d; ++k) {
        const float dk = b.cen[k] - a.cen[k];
        if (fabsf(dk) > bv) {
            bv = fabsf(dk);
            best = k;
            bs = dk;
        }
    }
    return a.rep[2 * best + (bs >= 0.f ? 1 : 0)];
}

// The 16 features of the ordered pair (a, b), rounded to FP16.
// ma, mb: core counts; na, nb: grid sizes; off: offset of Eq. (2);
// pa, pb: the two starting candidates' coordinates.
__device__ inline void pair_features(const CellSummary& A, const CellSummary& B, int d, double eps, uint32_t ma,
                                     uint32_t mb, uint32_t na, uint32_t nb, int off, const int32_t* pa,
                                     const int32_t* pb, float (&f)[kFeat]) {
    const float inv = (float)(1.0 / eps);
    float dc2 = 0.f, gap2 = 0.f, ea2 = 0.f, eb2 = 0.f, pp2 = 0.f, pab2 = 0.f, pba2 = 0.f;
    float dcv[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < d; ++k) {
        const float dc = B.cen[k] - A.cen[k];
        dc2 += dc * dc;
        if (k < 3) dcv[k] = dc;
        const float g = (float)max(max(B.lo[k] - A.hi[k], A.lo[k] - B.hi[k]), 0);
        gap2 += g * g;
        const float ea = (float)(A.hi[k] - A.lo[k]), eb = (float)(B.hi[k] - B.lo[k]);
        ea2 += ea * ea;
        eb2 += eb * eb;
        const float dp = (float)(pb[k] - pa[k]);
        pp2 += dp * dp;
        const float t1 = (float)pa[k] - B.cen[k], t2 = (float)pb[k] - A.cen[k];
        pab2 += t1 * t1;
        pba2 += t2 * t2;
    }
    const float la = log2f(1.f + (float)ma), lb = log2f(1.f + (float)mb);
    f[0] = la * (1.f / 16.f);
    f[1] = lb * (1.f / 16.f);
    f[2] = (float)off / (float)d;
    f[3] = sqrtf(dc2) * inv;
    f[4] = dcv[0] * inv;
    f[5] = dcv[1] * inv;
    f[6] = dcv[2] * inv;
    f[7] = sqrtf(gap2) * inv;
    f[8] = sqrtf(ea2) * inv;
    f[9] = sqrtf(eb2) * inv;
    f[10] = sqrtf(pp2) * inv;
    f[11] = sqrtf(pab2) * inv;
    f[12] = sqrtf(pba2) * inv;
    f[13] = (float)ma / (float)max(na, 1u);
    f[14] = (float)mb / (float)max(nb, 1u);
    f[15] = (la - lb) * (1.f / 8.f);
#pragma unroll
    for (int k = 0; k < kFeat; ++k) f[k] = __half2float(__float2half(f[k]));
}

// Offset of Eq. (2) between grids a and b (identifier rows 1..D).
__device__ inline int grid_offset(const GridView& g, uint32_t a, uint32_t b, int d) {
    int off = 0;
    for (int k = 1; k <= d; ++k) {
        const int dk = abs(g.ck[(int64_t)k * g.ck_stride + a] - g.ck[(int64_t)k * g.ck_stride + b]) - 1;
        off += dk > 0 ? dk * dk : 0;
    }
    return off;
}

// Features of the ordered pair (a, b) of core grids, plus both starting
// candidates.  Every lane computes the same values.
template <int D>
__device__ inline void pair_setup(const GridView& gv, const CoreOut& co, const CellSummary* sum, uint32_t a,
                                  uint32_t b, double eps, float (&f)[kFeat], uint32_t& rep_a, uint32_t& rep_b) {
    const CellSummary& A = sum[a];
    const CellSummary& B = sum[b];
    rep_a = rep_towards(A, B, D);
    rep_b = rep_towards(B, A, D);
    const uint32_t ba = co.core_begin[a], ma = co.core_cnt[a];
    const uint32_t bb = co.core_begin[b], mb = co.core_cnt[b];
    const uint32_t na = gv.cell_start[a + 1] - gv.cell_start[a];
    const uint32_t nb = gv.cell_start[b + 1] - gv.cell_start[b];
    int32_t pa[kMaxD] = {}, pb[kMaxD] = {};
    {
        int32_t ta[D], tb[D];
        load_row<D>(co.ccrd, ba + rep_a, ta);
        load_row<D>(co.ccrd, bb + rep_b, tb);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            pa[k] = ta[k];
            pb[k] = tb[k];
        }
    }
    pair_features(A, B, D, eps, ma, mb, na, nb, grid_offset(gv, a, b, D), pa, pb, f);
}

}  // namespace gd
