// FastMerging (Algorithms 4-5) on one pair with a whole workgroup of NW
// waves, for core sets large enough that one wave's serial scans would leave
// the GPU idle (a few hundred grids of 1e4-1e5 core points, as 2-D data with
// a large eps produces).  The steps and their order are those of
// fast_merging_from (fastmerge.hpp): each nearest-point search and each
// Pruning pass is split over the waves word by word (wave w takes bitmap
// words w, w + NW, ...), and the per-wave results are combined in LDS, so
// every bitmap, every nearest point (ties to the lowest position) and the
// answer are the same as on one wave.  Every decision is taken from
// combined values, so all threads of the workgroup follow the same control
// flow and every barrier is reached by all of them.  The bitmaps live in
// device memory (one slab per workgroup); a word is written only by the
// wave that owns it, and the barriers (workgroup-scope fences) order those
// writes before other waves read them.
#pragma once

#include "fastmerge.hpp"

namespace gd {

template <int D, int NW>
struct BlockScratch {
    uint64_t key[NW];   // per wave: smallest distance
    uint32_t pos[NW];   // and the lowest position holding it
    int32_t row[NW][D];
    float cmin[NW];
    uint32_t flag[NW];
};

template <int D, bool kWide, int NW>
__device__ __forceinline__ typename Dist<kWide>::T block_nearest(const PointSet& s, const int32_t (&p)[D],
                                                                 unsigned long long& ndist, int32_t (&row)[D],
                                                                 BlockScratch<D, NW>& sh) {
    const int lane = lane_id(), w = wave_id();
    uint64_t best = ~0ull;
    uint32_t bpos = ~0u;
    int32_t br[D];
#pragma unroll
    for (int k = 0; k < D; ++k) br[k] = 0;
    for (uint32_t wd = (uint32_t)w; wd < s.words; wd += NW) {
        const uint64_t mk = s.alive[wd];
        if (!mk) continue;
        ndist += (unsigned long long)popc64(mk);
        if ((mk >> lane) & 1ull) {
            int32_t y[D];
            load_point<D>(s, wd * kWave + lane, y);
            typename Dist<kWide>::T dd = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) dd += sqd<kWide>(y[k], p[k]);
            if ((uint64_t)dd < best) {  // later words of this lane hold larger positions
                best = dd;
                bpos = wd * kWave + lane;
#pragma unroll
                for (int k = 0; k < D; ++k) br[k] = y[k];
            }
        }
    }
    const uint64_t m = wave_min_u64(best);
    const uint32_t pm = wave_min_u32(best == m ? bpos : ~0u);
    if (lane == 0) {
        sh.key[w] = m;
        sh.pos[w] = pm;
    }
    if (pm != ~0u && lane == (int)(pm & (uint32_t)(kWave - 1))) {
#pragma unroll
        for (int k = 0; k < D; ++k) sh.row[w][k] = br[k];
    }
    __syncthreads();
    uint64_t bm = ~0ull;
    uint32_t bp = ~0u;
    int bw = 0;
#pragma unroll
    for (int v = 0; v < NW; ++v) {
        const uint64_t km = sh.key[v];
        const uint32_t kp = sh.pos[v];
        if (km < bm || (km == bm && kp < bp)) {
            bm = km;
            bp = kp;
            bw = v;
        }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) row[k] = sh.row[bw][k];
    __syncthreads();
    return (typename Dist<kWide>::T)bm;
}

// Pruning (Algorithm 4), the same tests as pruning() in fastmerge.hpp.
template <int D, bool kWide, int NW>
__device__ __forceinline__ bool block_pruning(const PointSet& a, const PointSet& b, const int32_t (&p)[D],
                                              const int32_t (&q)[D], typename Dist<kWide>::T dpq,
                                              typename Dist<kWide>::T T, double eps_d, unsigned long long& ndist,
                                              BlockScratch<D, NW>& sh) {
    using DT = typename Dist<kWide>::T;
    const int lane = lane_id(), w = wave_id();
    int32_t pq[D];
#pragma unroll
    for (int k = 0; k < D; ++k) pq[k] = q[k] - p[k];
    const float eps = (float)eps_d;
    const float a2 = (float)dpq;
    const float rna = __builtin_amdgcn_rsqf(a2);  // 1 / |pq|
    // lambda over the live points of b, each wave over its words
    float cmin = 2.f;
    bool off = false;
    for (uint32_t wd = (uint32_t)w; wd < b.words; wd += NW) {
        const uint64_t mk = b.alive[wd];
        if (!mk) continue;
        ndist += (unsigned long long)popc64(mk);
        if (!((mk >> lane) & 1ull)) continue;
        int32_t y[D];
        load_point<D>(b, wd * kWave + lane, y);
        int32_t py[D];
        int64_t dot = 0;
        DT b2 = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            py[k] = y[k] - p[k];
            dot += (int64_t)pq[k] * py[k];
            b2 += sqd<kWide>(y[k], p[k]);
        }
        const float dotf = (float)dot;
        const float h2 = (float)(b2 - T);
        if (dot < 0 && dotf * dotf >= a2 * h2 * (1.f - 1e-3f)) {
            off = true;
        } else {
            float cross = 0.f;
#pragma unroll
            for (int k = 0; k < D; ++k)
#pragma unroll
                for (int l = k + 1; l < D; ++l) {
                    const float mnr = (float)((int64_t)pq[k] * py[l] - (int64_t)pq[l] * py[k]);
                    cross += mnr * mnr;
                }
            const float num = dotf * __builtin_amdgcn_sqrtf(h2) - eps * __builtin_amdgcn_sqrtf(cross);
            const float c = num * rna * __builtin_amdgcn_rcpf((float)b2);
            cmin = c < cmin ? c : cmin;
        }
    }
    const bool off_w = ballot(off) != 0;
    const float cmin_w = wave_min_f32(cmin);
    if (lane == 0) {
        sh.cmin[w] = cmin_w;
        sh.flag[w] = off_w ? 1u : 0u;
    }
    __syncthreads();
    float cm = 2.f;
    bool of = false;
#pragma unroll
    for (int v = 0; v < NW; ++v) {
        cm = sh.cmin[v] < cm ? sh.cmin[v] : cm;
        of = of || sh.flag[v] != 0u;
    }
    __syncthreads();
    const float thr = cm - kAngleMargin;
    uint64_t any = 0;
    for (uint32_t wd = (uint32_t)w; wd < a.words; wd += NW) {
        const uint64_t mk = a.alive[wd];
        if (!mk) continue;
        ndist += (unsigned long long)popc64(mk);
        bool keep = false;
        if ((mk >> lane) & 1ull) {
            int32_t x[D];
            load_point<D>(a, wd * kWave + lane, x);
            DT ax = 0;
            int64_t dotx = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                ax += sqd<kWide>(x[k], p[k]);
                dotx += (int64_t)pq[k] * (x[k] - p[k]);
            }
            const int64_t s = (int64_t)dpq - (int64_t)T - (int64_t)ax;
            bool tri;
            if constexpr (kWide)
                tri = s > 0 && (unsigned __int128)4 * T * ax < (unsigned __int128)s * (uint64_t)s;
            else
                tri = s > 0 && (uint64_t)4 * (uint64_t)T * (uint64_t)ax < (uint64_t)s * (uint64_t)s;
            keep = !tri;
            if (keep && !of && ax > 0) {
                const float cth = (float)dotx * rna * __builtin_amdgcn_rsqf((float)ax);
                if (cth < thr) keep = false;
            }
        }
        const uint64_t nm = ballot(keep);
        if (lane == 0) a.alive[wd] = nm;
        any |= nm;
    }
    if (lane == 0) sh.flag[w] = any != 0 ? 1u : 0u;
    __syncthreads();
    bool any_all = false;
#pragma unroll
    for (int v = 0; v < NW; ++v) any_all = any_all || sh.flag[v] != 0u;
    __syncthreads();
    return any_all;
}

template <int NW>
__device__ __forceinline__ void block_init_alive(const PointSet& s) {
    const int lane = lane_id(), w = wave_id();
    for (uint32_t wd = (uint32_t)w; wd < s.words; wd += NW) {
        const uint32_t rem = s.m - wd * kWave;
        if (lane == 0) s.alive[wd] = rem >= (uint32_t)kWave ? ~0ull : ((1ull << rem) - 1ull);
    }
}

// Algorithm 5 from P0 (a point of si) on the workgroup: 1 (yes), 0 (no) or
// -1 (iteration bound exceeded), the same in every thread.
template <int D, bool kWide, int NW>
__device__ int fast_merging_block(PointSet si, PointSet sj, const int32_t (&P0)[D], typename Dist<kWide>::T T,
                                  typename Dist<kWide>::T Tyes, double eps, unsigned long long& ndist,
                                  uint32_t& iters, BlockScratch<D, NW>& sh) {
    using DT = typename Dist<kWide>::T;
    block_init_alive<NW>(si);
    block_init_alive<NW>(sj);
    __syncthreads();
    const uint32_t bound = si.m + sj.m + 2;
    int32_t P[D], Q[D];
#pragma unroll
    for (int k = 0; k < D; ++k) P[k] = P0[k];
    for (iters = 1;; ++iters) {
        if (iters > bound) return -1;
        const DT dq = block_nearest<D, kWide, NW>(sj, P, ndist, Q, sh);
        if (dq <= Tyes) return 1;
        if (!block_pruning<D, kWide, NW>(si, sj, P, Q, dq, T, eps, ndist, sh)) return 0;
        const DT dp = block_nearest<D, kWide, NW>(si, Q, ndist, P, sh);
        if (dp <= Tyes) return 1;
        if (!block_pruning<D, kWide, NW>(sj, si, Q, P, dp, T, eps, ndist, sh)) return 0;
    }
}

}  // namespace gd
