// Learned proposal: per-grid summaries, harvesting of training pairs from
// the method's own merge decisions, FP16 training (FP32 accumulation and
// master weights) and FP16 inference of the pair scorer.
#include "fastmerge.hpp"
#include "learned.hpp"

namespace gd {

// ---------------------------------------------------------------- summaries
// One wave per core grid: centroid, bounding box and the positions of the
// extreme core points along every axis, over a sample of at most 64 core
// points (the features only guide the merge; any core point may start it).
template <int D>
__global__ __launch_bounds__(kBlock) void summary_kernel(GridView gv, CoreOut co, CellSummary* __restrict__ out) {
    const int lane = lane_id();
    const int64_t c = block_id() * kWavesPerBlock + wave_id();
    if (c >= (int64_t)*gv.ncell_dev || c >= gv.ncell) return;  // out[] holds gv.ncell summaries
    const uint32_t b = co.core_begin[c], m = co.core_cnt[c];
    if (m == 0) return;
    // coordinates are below 2^25 (minus the instance minimum, |x| <= 2^24),
    // so value << 6 | position fits 32 bits and 64 of them sum exactly
    uint32_t sum[D], lo[D], hi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        sum[k] = 0u;
        lo[k] = ~0u;
        hi[k] = 0u;
    }
    // the first (at most) 64 core points: in input order within the grid, a
    // uniform sample of its core set
    const uint32_t ms = min(m, (uint32_t)kWave);
    if ((uint32_t)lane < ms) {
        int32_t p[D];
        load_row<D>(co.ccrd, b + lane, p);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const uint32_t v = (uint32_t)p[k];
            sum[k] = v;
            lo[k] = (v << 6) | (uint32_t)lane;          // smallest value, lowest position
            hi[k] = (v << 6) | (uint32_t)(63 - lane);   // largest value, lowest position
        }
    }
    CellSummary s;
#pragma unroll
    for (int k = 0; k < kMaxD; ++k) {
        s.cen[k] = 0.f;
        s.lo[k] = s.hi[k] = 0;
        s.rep[2 * k] = s.rep[2 * k + 1] = 0;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const uint32_t tot = wave_sum(sum[k]);
        const uint32_t l = ~wave_max_u32(~lo[k]);
        const uint32_t h = wave_max_u32(hi[k]);
        s.cen[k] = (float)((double)tot / (double)ms);
        s.lo[k] = (int32_t)(l >> 6);
        s.hi[k] = (int32_t)(h >> 6);
        s.rep[2 * k] = l & 63u;
        s.rep[2 * k + 1] = 63u - (h & 63u);
    }
    if (lane == 0) out[c] = s;
}

hipError_t launch_summaries(const GridView& g, const CoreOut& c, CellSummary* out, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    GD_DISPATCH_D(g.D, (summary_kernel<D><<<grid_of(grid_for(g.ncell, kWavesPerBlock)), dim3(kBlock), 0, st>>>(g, c,
                                                                                                          out)));
    return hipGetLastError();
}

// ------------------------------------------------------------------ harvest
// Training pairs from the last clustering: core grid pairs (a, b), a < b,
// sampled by a hash of the pair.  For each, FastMerging runs three times:
// from a's first core point (the plain method), from a's and from b's
// candidate towards the other grid.  Targets: merge answer, whether starting
// from b costs fewer distance evaluations, and whether the sides differ.
template <int D>
__global__ __launch_bounds__(kBlock) void harvest_kernel(GridView gv, CoreOut co, const CellSummary* __restrict__ sum,
                                                         const uint64_t* __restrict__ nei_off,
                                                         const uint32_t* __restrict__ nei, uint32_t seed,
                                                         uint32_t keep_mod, int64_t cap, uint32_t words,
                                                         __half* __restrict__ X, float* __restrict__ Tg,
                                                         float* __restrict__ C, unsigned long long* counter) {
    extern __shared__ uint64_t smem[];
    const int lane = lane_id();
    const int w = wave_id();
    const int64_t a = block_id() * kWavesPerBlock + w;
    if (a >= (int64_t)*gv.ncell_dev) return;
    const uint32_t ba = co.core_begin[a], ma = co.core_cnt[a];
    if (ma == 0 || ma > 64u * words) return;
    const Inst& I = cell_inst(gv, a);
    const double eps = (double)I.eps;
    uint64_t* bits_a = smem + (int64_t)w * 2 * words;
    uint64_t* bits_b = bits_a + words;
    const uint64_t e0 = nei_off[a], e1 = nei_off[a + 1];
    for (uint64_t e = e0; e < e1; e += kWave) {
        const uint64_t idx = e + lane;
        uint32_t cb = 0;
        bool take = false;
        if (idx < e1) {
            cb = nei[idx];
            if (cb > (uint32_t)a) {
                const uint32_t mb = co.core_cnt[cb];
                uint32_t h = (uint32_t)a * 0x9E3779B1u ^ (cb + seed) * 0x85EBCA77u;
                h ^= h >> 15;
                h *= 0xC2B2AE3Du;
                h ^= h >> 13;
                take = mb > 0 && mb <= 64u * words && (h % keep_mod) == 0;
            }
        }
        uint64_t todo = ballot(take);
        while (todo) {
            const int l = ffs64(todo);
            todo &= todo - 1ull;
            const uint32_t b = readlane(cb, l);
            unsigned long long slot = 0;
            if (lane == 0) slot = atomicAdd(counter, 1ull);
            slot = (unsigned long long)__shfl((long long)slot, 0);
            if ((int64_t)slot >= cap) return;
            float f[kFeat];
            uint32_t ra, rb;
            pair_setup<D>(gv, co, sum, (uint32_t)a, b, eps, f, ra, rb);
            const uint32_t bb = co.core_begin[b], mb = co.core_cnt[b];
            PointSet sa{co.ccrd, ba, ma, bits_a, (ma + kWave - 1) / kWave};
            PointSet sb{co.ccrd, bb, mb, bits_b, (mb + kWave - 1) / kWave};
            unsigned long long c0 = 0, c1 = 0, c2 = 0;
            uint32_t it;
            const int y = fast_merging<D>(sa, sb, 0u, I.T, I.T, eps, c0, it);
            fast_merging<D>(sa, sb, ra, I.T, I.T, eps, c1, it);
            fast_merging<D>(sb, sa, rb, I.T, I.T, eps, c2, it);
            if (lane < kFeat) {
                float v = 0.f;
#pragma unroll
                for (int k = 0; k < kFeat; ++k) v = (k == lane) ? f[k] : v;
                X[slot * kFeat + lane] = __float2half(v);
            }
            if (lane == 0) {
                Tg[slot * 3 + 0] = y > 0 ? 1.f : 0.f;
                Tg[slot * 3 + 1] = c2 < c1 ? 1.f : 0.f;
                Tg[slot * 3 + 2] = c2 != c1 ? 1.f : 0.f;
                if (C) {
                    C[slot * 3 + 0] = (float)c0;
                    C[slot * 3 + 1] = (float)c1;
                    C[slot * 3 + 2] = (float)c2;
                }
            }
        }
    }
}

hipError_t launch_harvest(const GridView& g, const CoreOut& c, const CellSummary* sum, const uint64_t* nei_off,
                          const uint32_t* nei, uint32_t seed, uint32_t keep_mod, int64_t cap, int64_t max_core,
                          __half* X, float* Tg, float* C, unsigned long long* counter, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    const uint32_t words = (uint32_t)((std::min<int64_t>(max_core, 16384) + kWave - 1) / kWave);
    const size_t lds = (size_t)kWavesPerBlock * 2 * words * sizeof(uint64_t);
    GD_DISPATCH_D(g.D, (harvest_kernel<D><<<grid_of(grid_for(g.ncell, kWavesPerBlock)), dim3(kBlock), lds, st>>>(
                           g, c, sum, nei_off, nei, seed, keep_mod, cap, words, X, Tg, C, counter)));
    return hipGetLastError();
}

// ---------------------------------------------------------------- inference
// One wave per sample: z [B x 2] for features X [B x 16] (FP16).
__global__ __launch_bounds__(kBlock) void mlp_forward_kernel(const __half* __restrict__ X, int64_t B,
                                                             const __half* __restrict__ params, float* __restrict__ Z) {
    __shared__ MlpMfma W;
    __shared__ MlpMfmaScratch S[kWavesPerBlock];
    mlp_mfma_load(W, params);
    __syncthreads();
    const int w = wave_id(), l = lane_id();
    const int64_t stride = (int64_t)gridDim.x * kWavesPerBlock * 16;
    for (int64_t r0 = ((int64_t)blockIdx.x * kWavesPerBlock + w) * 16; r0 < B; r0 += stride) {
        for (int i = l; i < 16 * kFeat; i += kWave) {
            const int row = i / kFeat, k = i % kFeat;
            S[w].feat[row][k] = r0 + row < B ? (_Float16)__half2float(X[(r0 + row) * kFeat + k]) : (_Float16)0.f;
        }
        wave_sync();
        float z0[4], z1[4];
        mlp_forward_mfma(W, S[w], z0, z1);
        if ((l & 15) == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t row = r0 + 4 * (l >> 4) + j;
                if (row < B) {
                    Z[row * 2 + 0] = z0[j];
                    Z[row * 2 + 1] = z1[j];
                }
            }
        }
    }
}

hipError_t launch_mlp_forward(const __half* X, int64_t B, const __half* params, float* Z, hipStream_t st) {
    if (B <= 0) return hipSuccess;
    int64_t blocks = (B + 16 * kWavesPerBlock - 1) / (16 * kWavesPerBlock);
    if (blocks > 2048) blocks = 2048;
    mlp_forward_kernel<<<dim3((unsigned)blocks), dim3(kBlock), 0, st>>>(X, B, params, Z);
    return hipGetLastError();
}

// ----------------------------------------------------------------- training
__device__ __forceinline__ float softplusf(float z) { return z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z)); }
__device__ __forceinline__ float sigmoidf(float z) { return 1.f / (1.f + expf(-z)); }

// One workgroup of four waves.  Each step: round the master weights to FP16
// (kept widened in LDS), every wave runs forward + backward for its share of
// the batch with one lane per hidden unit, accumulating its gradient rows in
// registers (FP32); the rows are summed in LDS, then an Adam update.
__global__ __launch_bounds__(kBlock) void mlp_train_kernel(TrainArgs a) {
    __shared__ MlpLds W;
    __shared__ float G[kParams];
    __shared__ float hbuf[kWavesPerBlock][kWave];
    __shared__ float dbuf[kWavesPerBlock][kWave];
    __shared__ float s_loss;
    const int tid = threadIdx.x, w = wave_id(), u = lane_id();
    const float inv_b = 1.f / (float)a.batch;
    for (int step = 0; step < a.steps; ++step) {
        for (int i = tid; i < kParams; i += kBlock) {
            G[i] = 0.f;
            const float v = __half2float(__float2half(a.params[i]));
            if (i < oB1) W.w1t[(i - oW1) % kFeat][(i - oW1) / kFeat] = v;
            else if (i < oW2) W.b1[i - oB1] = v;
            else if (i < oB2) W.w2t[(i - oW2) % kHid][(i - oW2) / kHid] = v;
            else if (i < oW3) W.b2[i - oB2] = v;
            else if (i < oB3) W.w3[(i - oW3) / kHid][(i - oW3) % kHid] = v;
            else W.b3[i - oB3] = v;
        }
        if (tid == 0) s_loss = 0.f;
        __syncthreads();
        float gW1[kFeat], gW2[kHid], gb1 = 0.f, gb2 = 0.f, gW30 = 0.f, gW31 = 0.f, gb30 = 0.f, gb31 = 0.f;
#pragma unroll
        for (int k = 0; k < kFeat; ++k) gW1[k] = 0.f;
#pragma unroll
        for (int k = 0; k < kHid; ++k) gW2[k] = 0.f;
        float lsum = 0.f;
        for (int r = w; r < a.batch; r += kWavesPerBlock) {
            const int64_t s = a.order[(int64_t)step * a.batch + r];
            float f[kFeat];
#pragma unroll
            for (int k = 0; k < kFeat; ++k) f[k] = __half2float(a.x[s * kFeat + k]);
            const float y0 = a.t[s * 3 + 0], y1 = a.t[s * 3 + 1], w1 = a.t[s * 3 + 2];
            const MlpTrace tr = mlp_forward_wave(W, f, hbuf[w]);
            // hbuf[w] still holds h1 (mlp_forward_wave does not clear it)
            lsum += softplusf(tr.z0) - y0 * tr.z0 + kLambda * w1 * (softplusf(tr.z1) - y1 * tr.z1);
            const float dz0 = (sigmoidf(tr.z0) - y0) * inv_b;
            const float dz1 = kLambda * w1 * (sigmoidf(tr.z1) - y1) * inv_b;
            gW30 += dz0 * tr.h2;
            gW31 += dz1 * tr.h2;
            gb30 += dz0;
            gb31 += dz1;
            const float da2 = (tr.a2 > 0.f) ? (W.w3[0][u] * dz0 + W.w3[1][u] * dz1) : 0.f;
            gb2 += da2;
#pragma unroll
            for (int k = 0; k < kHid; ++k) gW2[k] += da2 * hbuf[w][k];
            dbuf[w][u] = da2;
            wave_sync();
            float dh1 = 0.f;
#pragma unroll 8
            for (int v = 0; v < kHid; ++v) dh1 += W.w2t[u][v] * dbuf[w][v];
            const float da1 = (tr.a1 > 0.f) ? dh1 : 0.f;
            gb1 += da1;
#pragma unroll
            for (int k = 0; k < kFeat; ++k) gW1[k] += da1 * f[k];
            wave_sync();
        }
        // the waves add their rows in wave order (a fixed summation order,
        // so the gradient of a batch is the same on every call); within a
        // wave every lane owns its own addresses
        for (int turn = 0; turn < kWavesPerBlock; ++turn) {
            if (w == turn) {
#pragma unroll
                for (int k = 0; k < kFeat; ++k) G[oW1 + u * kFeat + k] += gW1[k];
                G[oB1 + u] += gb1;
#pragma unroll
                for (int k = 0; k < kHid; ++k) G[oW2 + u * kHid + k] += gW2[k];
                G[oB2 + u] += gb2;
                G[oW3 + u] += gW30;
                G[oW3 + kHid + u] += gW31;
                if (u == 0) {
                    G[oB3] += gb30;
                    G[oB3 + 1] += gb31;
                    s_loss += lsum;
                }
            }
            __syncthreads();
        }
        if (a.grad && step == 0)
            for (int i = tid; i < kParams; i += kBlock) a.grad[i] = G[i];
        if (a.loss && tid == 0) a.loss[step] = s_loss * inv_b;
        if (a.update) {
            // Adam (beta1 0.9, beta2 0.999, eps 1e-8).  The step's bias
            // corrections 1 - beta^t are taken in double (in single precision
            // 1 - 0.999^t loses five digits to cancellation), and 1 - beta
            // is the single-precision value of the exact difference.
            const int t = a.adam_t0 + step + 1;
            const double c1 = 1.0 - pow(0.9, (double)t), c2 = 1.0 - pow(0.999, (double)t);
            const float inv_c1 = (float)(1.0 / c1), inv_sqrt_c2 = (float)(1.0 / sqrt(c2));
            const float b1 = 0.9f, b2 = 0.999f, omb1 = 0.1f, omb2 = 0.001f;
            for (int i = tid; i < kParams; i += kBlock) {
                const float g = G[i];
                const float mm = b1 * a.m[i] + omb1 * g;
                const float vv = b2 * a.v[i] + omb2 * (g * g);
                a.m[i] = mm;
                a.v[i] = vv;
                a.params[i] -= a.lr * (mm * inv_c1) / (sqrtf(vv) * inv_sqrt_c2 + 1e-8f);
            }
        }
        __syncthreads();
    }
    if (a.blob)
        for (int i = tid; i < kParams; i += kBlock) a.blob[i] = __float2half(a.params[i]);
}

hipError_t launch_mlp_train(const TrainArgs& a, hipStream_t st) {
    mlp_train_kernel<<<1, kBlock, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace gd
