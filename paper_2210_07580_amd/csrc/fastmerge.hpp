// FastMerging (Algorithm 5) with Pruning (Algorithm 4) on a wave, and the
// lock-free union-find over core grids, shared by the merge, harvesting and
// test kernels.
//
// One wave per core grid g_i, in LDF order.  For each core grid g_j in
// Nei(g_i) that comes later in that order (so every unordered pair is tested
// once, by its lower-density grid) the wave skips the pair if find(i) ==
// find(j) and otherwise decides MinDist(s_i, s_j) <= eps with FastMerging;
// on "yes" it unions the two sets.  Union-find is lock-free: a root's parent
// moves only from itself to a smaller grid index by compare-and-swap, and
// find() halves paths; every root is its component's smallest grid index.
//
// FastMerging on a wave: s_i and s_j are contiguous runs of the compacted
// core-point arrays; the points still in each set are a bitmap in LDS, one
// 64-bit word per 64 points, so a word is exactly one wave's ballot.
//   nearest(p, s_j): each lane evaluates one live point per word, then a
//     wave min over (squared distance << 32 | position) gives argmin with
//     ties to the lowest position.
//   Pruning(s_a, s_b, p, q), with a = D(p, q) > eps^2:
//     triangle rule, exactly in integers: drop x when
//       dist(x,p) < dist(p,q) - eps  <=>  s = a - eps^2 - D(x,p) > 0 and
//                                         4 eps^2 D(x,p) < s^2
//     angle rule (Definition 7, Theorem 1) in the cosine domain: with
//       b = |py|, cos(alpha) = sqrt(b^2 - eps^2)/b, sin(alpha) = eps/b,
//       cos(beta) = pq.py/(|pq| b), sin(beta) from the exact cross terms,
//       cos(lambda_y) = (pq.py sqrt(b^2 - eps^2) - eps |pq x py|) / (|pq| b^2)
//     lambda = max_y lambda_y, i.e. cos(lambda) = min_y cos(lambda_y); if
//     some lambda_y reaches pi the rule is switched off for this call.
//     The cosines are evaluated in single precision and x is dropped when
//     cos(theta_x) < cos(lambda) - 1e-4: the margin is far above the
//     rounding of these terms (see kAngleMargin), so rounding can only keep
//     a point, never drop one wrongly, and the answer stays exact (Theorem 2).
//   The start point p is the first core point of the larger of the two sets
//   (the paper picks a point of s_i at random; the choice does not change
//   the answer), so that the first nearest-point search, which on a yes is
//   the only one, runs over the smaller set.  If a Pruning call
//   empties a set the answer is "no" at once.
//   Wide path (eps above the 32-bit bound): squared distances in 64 bits,
//   the triangle rule's products in 128 bits, and the same single-precision
//   cosines (their error bound is relative, so larger operands keep it).
//   Approximate FastMerging (the remark on numerical error, Section 4.3.3):
//   the two "yes" tests accept D(p, q) <= Tyes = (eps + delta)^2 while
//   Pruning keeps eps; then every pair with MinDist <= eps still answers yes,
//   and a yes implies MinDist <= eps + delta.  Tyes = eps^2 is the exact test.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace gd {

// Root of x's set, given p, a value parent[x] has held (a caller may load it
// early, beside other loads).  Links only ever point closer to a root, so a
// stale p still leads to the current root.  Path halving on the way; a
// parent found to be its own parent is returned without loading it again.
__device__ __forceinline__ uint32_t uf_find_at(uint32_t* parent, uint32_t x, uint32_t p) {
    for (;;) {
        if (p == x) return x;
        const uint32_t gp = load_acq(&parent[p]);
        if (gp == p) return p;
        store_rel(&parent[x], gp);
        x = gp;
        p = load_acq(&parent[x]);
    }
}

__device__ __forceinline__ uint32_t uf_find(uint32_t* parent, uint32_t x) {
    return uf_find_at(parent, x, load_acq(&parent[x]));
}

__device__ __forceinline__ void uf_union(uint32_t* parent, uint32_t a, uint32_t b) {
    for (;;) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return;
        if (a > b) {
            const uint32_t t = a;
            a = b;
            b = t;
        }
        if (atomicCAS(&parent[b], b, a) == b) return;
    }
}

// Union given ra and rb, nodes on the root paths of the two elements (their
// roots as last seen).  The common case is one compare-and-swap: the larger
// of the two is still a root and goes under the smaller, which keeps every
// root the smallest index of its component.  Otherwise both are resolved
// again.  Returns the root the sets were joined under (as it stood then);
// callers use it as a hint: a later find() that returns it proves the
// connection, a stale hint only costs an extra exact test.
__device__ __forceinline__ uint32_t uf_union_from(uint32_t* parent, uint32_t ra, uint32_t rb) {
    for (;;) {
        if (ra == rb) return ra;
        const uint32_t a = ra < rb ? ra : rb;
        const uint32_t b = ra < rb ? rb : ra;
        if (atomicCAS(&parent[b], b, a) == b) return a;
        ra = uf_find(parent, a);
        rb = uf_find(parent, b);
    }
}

// A run of point rows (row_stride(D) int32 each): position i is row base + i.
struct PointSet {
    const int32_t* rows;
    uint32_t base;        // first row of the set
    uint32_t m;           // size
    uint64_t* alive;      // LDS bitmap, ceil(m / 64) words
    uint32_t words;
};

template <int D>
__device__ __forceinline__ void load_point(const PointSet& s, uint32_t pos, int32_t (&x)[D]) {
    load_row<D>(s.rows, (int64_t)s.base + pos, x);
}

constexpr uint32_t kUnroll = 2;  // words of a set whose loads are issued together

// Loads the point of this lane in word w (position clamped into the set so
// the address is always valid; callers ignore lanes whose bit is clear).
template <int D>
__device__ __forceinline__ void load_lane_point(const PointSet& s, uint32_t w, int32_t (&x)[D]) {
    uint32_t pos = w * kWave + lane_id();
    pos = pos < s.m ? pos : s.m - 1;
    load_point<D>(s, pos, x);
}

// argmin over live y of D(p, y): returns that distance, and the winning
// point's row in `row` (from the winning lane's registers: no second load
// of it); ties go to the lowest position.  s must hold a live point.  The
// 32-bit path ranks (D << 32 | position) in one wave minimum; the wide path
// takes the minimum distance, then the lowest position holding it.
template <int D, bool kWide = false>
__device__ __forceinline__ typename Dist<kWide>::T nearest(const PointSet& s, const int32_t (&p)[D],
                                                           unsigned long long& ndist, int32_t (&row)[D]) {
    const int lane = lane_id();
    if constexpr (kWide) {
        uint64_t best = ~0ull;
        uint32_t bpos = ~0u;
        int32_t br[D];
#pragma unroll
        for (int k = 0; k < D; ++k) br[k] = 0;
        for (uint32_t w = 0; w < s.words; ++w) {
            const uint64_t mk = s.alive[w];
            if (!mk) continue;
            ndist += (unsigned long long)popc64(mk);
            if ((mk >> lane) & 1ull) {
                int32_t y[D];
                load_point<D>(s, w * kWave + lane, y);
                uint64_t dd = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) dd += sqd<true>(y[k], p[k]);
                if (dd < best) {  // later words only hold larger positions
                    best = dd;
                    bpos = w * kWave + lane;
#pragma unroll
                    for (int k = 0; k < D; ++k) br[k] = y[k];
                }
            }
        }
        const uint64_t m = wave_min_u64(best);
        const uint32_t pos = wave_min_u32(best == m ? bpos : ~0u);
        const int wl = __builtin_amdgcn_readfirstlane((int)(pos & (uint32_t)(kWave - 1)));
#pragma unroll
        for (int k = 0; k < D; ++k) row[k] = readlane(br[k], wl);
        return m;
    } else {
    uint64_t best = ~0ull;
    int32_t br[D];
#pragma unroll
    for (int k = 0; k < D; ++k) br[k] = 0;
    for (uint32_t w0 = 0; w0 < s.words; w0 += kUnroll) {
        uint64_t mk[kUnroll];
        int32_t y[kUnroll][D];
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
            const uint32_t w = w0 + u;
            mk[u] = w < s.words ? s.alive[w] : 0ull;
            if (mk[u]) load_lane_point<D>(s, w, y[u]);
        }
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
            ndist += (unsigned long long)popc64(mk[u]);
            if ((mk[u] >> lane) & 1ull) {
                uint32_t dd = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) dd += sq24(y[u][k], p[k]);
                const uint64_t cand = ((uint64_t)dd << 32) | ((w0 + u) * kWave + lane);
                if (cand < best) {
                    best = cand;
#pragma unroll
                    for (int k = 0; k < D; ++k) br[k] = y[u][k];
                }
            }
        }
    }
    const uint64_t m = wave_min_u64(best);
    // position % 64 is the lane that found it
    const int wl = __builtin_amdgcn_readfirstlane((int)((uint32_t)m & (uint32_t)(kWave - 1)));
#pragma unroll
    for (int k = 0; k < D; ++k) row[k] = readlane(br[k], wl);
    return (uint32_t)(m >> 32);
    }
}

__device__ __forceinline__ float wave_min_f32(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const float t = __shfl_xor(v, o);
        v = t < v ? t : v;
    }
    return v;
}

// Rounding slack of the single-precision angle rule.  Every operand is an
// integer (coordinates, dot products, 2x2 minors, squared norms, all below
// 2^36) converted to float with relative error 2^-24, and square roots and
// reciprocals are within two ulps, so each computed cosine is within 1e-6 of
// the exact one (both terms of the cos(lambda_y) numerator are bounded by its
// denominator).  With a margin of 1e-4 a point is only dropped when the exact
// test drops it too.
constexpr float kAngleMargin = 1e-4f;

// Algorithm 4: remove from `a` the points that cannot be within eps of any
// live point of `b`, given anchor p in a and q = argmin_{y in b} D(p, y) with
// D(p, q) = dpq > T.  Returns whether `a` keeps any point.
template <int D, bool kWide = false>
__device__ __forceinline__ bool pruning(const PointSet& a, const PointSet& b, const int32_t (&p)[D],
                                        const int32_t (&q)[D], typename Dist<kWide>::T dpq,
                                        typename Dist<kWide>::T T, double eps_d, unsigned long long& ndist) {
    using DT = typename Dist<kWide>::T;
    const int lane = lane_id();
    int32_t pq[D];
#pragma unroll
    for (int k = 0; k < D; ++k) pq[k] = q[k] - p[k];
    const float eps = (float)eps_d;
    const float a2 = (float)dpq;
    const float rna = __builtin_amdgcn_rsqf(a2);  // 1 / |pq|
    // lambda over the live points of b
    float cmin = 2.f;
    bool off = false;
    for (uint32_t w0 = 0; w0 < b.words; w0 += kUnroll) {
        uint64_t mk[kUnroll];
        int32_t yy[kUnroll][D];
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
            const uint32_t w = w0 + u;
            mk[u] = w < b.words ? b.alive[w] : 0ull;
            if (mk[u]) load_lane_point<D>(b, w, yy[u]);
        }
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
            ndist += (unsigned long long)popc64(mk[u]);
            if (!((mk[u] >> lane) & 1ull)) continue;
            int32_t py[D];
            int64_t dot = 0;
            DT b2 = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                py[k] = yy[u][k] - p[k];
                dot += (int64_t)pq[k] * py[k];
                b2 += sqd<kWide>(yy[u][k], p[k]);
            }
            const float dotf = (float)dot;
            const float h2 = (float)(b2 - T);  // b^2 - eps^2 > 0 since b^2 >= dpq > T
            // lambda_y >= pi, or too close to tell: the rule is off for this call
            if (dot < 0 && dotf * dotf >= a2 * h2 * (1.f - 1e-3f)) {
                off = true;
            } else {
                float cross = 0.f;  // |pq|^2 |py|^2 - (pq.py)^2 as a sum of squared 2x2 minors
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
    }
    off = ballot(off) != 0;
    cmin = wave_min_f32(cmin);
    const float thr = cmin - kAngleMargin;
    uint64_t any = 0;
    for (uint32_t w0 = 0; w0 < a.words; w0 += kUnroll) {
        uint64_t mk[kUnroll];
        int32_t xx[kUnroll][D];
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
            const uint32_t w = w0 + u;
            mk[u] = w < a.words ? a.alive[w] : 0ull;
            if (mk[u]) load_lane_point<D>(a, w, xx[u]);
        }
#pragma unroll
        for (uint32_t u = 0; u < kUnroll; ++u) {
            if (!mk[u]) continue;
            ndist += (unsigned long long)popc64(mk[u]);
            bool keep = false;
            if ((mk[u] >> lane) & 1ull) {
                DT ax = 0;
                int64_t dotx = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    ax += sqd<kWide>(xx[u][k], p[k]);
                    dotx += (int64_t)pq[k] * (xx[u][k] - p[k]);
                }
                const int64_t s = (int64_t)dpq - (int64_t)T - (int64_t)ax;
                bool tri;
                if constexpr (kWide)  // 4 eps^2 D(x,p) and s^2 reach 2^117: 128-bit products
                    tri = s > 0 && (unsigned __int128)4 * T * ax < (unsigned __int128)s * (uint64_t)s;
                else
                    tri = s > 0 && (uint64_t)4 * (uint64_t)T * (uint64_t)ax < (uint64_t)s * (uint64_t)s;
                keep = !tri;
                if (keep && !off && ax > 0) {
                    const float cth = (float)dotx * rna * __builtin_amdgcn_rsqf((float)ax);
                    if (cth < thr) keep = false;
                }
            }
            const uint64_t nm = ballot(keep);
            if (lane == 0) a.alive[w0 + u] = nm;
            any |= nm;
        }
    }
    wave_sync();
    return any != 0;
}

template <int D>
__device__ __forceinline__ void init_alive(const PointSet& s) {
    for (uint32_t w = lane_id(); w < s.words; w += kWave) {
        const uint32_t rem = s.m - w * kWave;
        s.alive[w] = rem >= (uint32_t)kWave ? ~0ull : ((1ull << rem) - 1ull);
    }
}

// Algorithm 5 from P0, the start point of si (its row, which a caller
// testing several pairs from one si loads once).  Returns 1 (yes), 0 (no)
// or -1 (iteration bound exceeded).
template <int D, bool kWide = false>
__device__ int fast_merging_from(PointSet si, PointSet sj, const int32_t (&P0)[D], typename Dist<kWide>::T T,
                                 typename Dist<kWide>::T Tyes, double eps, unsigned long long& ndist,
                                 uint32_t& iters) {
    using DT = typename Dist<kWide>::T;
    init_alive<D>(si);
    init_alive<D>(sj);
    wave_sync();
    const uint32_t bound = si.m + sj.m + 2;
    // P: the current point of si (first the start point), Q: its nearest in sj
    int32_t P[D], Q[D];
#pragma unroll
    for (int k = 0; k < D; ++k) P[k] = P0[k];
    for (iters = 1;; ++iters) {
        if (iters > bound) return -1;
        const DT dq = nearest<D, kWide>(sj, P, ndist, Q);
        if (dq <= Tyes) return 1;
        if (!pruning<D, kWide>(si, sj, P, Q, dq, T, eps, ndist)) return 0;
        const DT dp = nearest<D, kWide>(si, Q, ndist, P);
        if (dp <= Tyes) return 1;
        if (!pruning<D, kWide>(sj, si, Q, P, dp, T, eps, ndist)) return 0;
    }
}

// Algorithm 5 from position `start` of si.
template <int D, bool kWide = false>
__device__ int fast_merging(PointSet si, PointSet sj, uint32_t start, typename Dist<kWide>::T T,
                            typename Dist<kWide>::T Tyes, double eps, unsigned long long& ndist, uint32_t& iters) {
    int32_t P0[D];
    load_point<D>(si, start, P0);
    return fast_merging_from<D, kWide>(si, sj, P0, T, Tyes, eps, ndist, iters);
}

}  // namespace gd
