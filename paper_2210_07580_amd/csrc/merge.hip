// Merging core grids (Section 4.3): FastMerging (Algorithm 5) with Pruning
// (Algorithm 4), and union-find over core grids visited in ascending
// core-count order (the LDF variant of Section 5.2).
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
//     x is dropped when cos(theta_x) < cos(lambda) - 1e-10: the margin is far
//     above the float64 rounding of these terms, so rounding can only keep a
//     point, never drop one wrongly, and the answer stays exact (Theorem 2).
//   The start point p is the first core point of s_i (the paper picks one at
//   random; the choice does not change the answer).  If a Pruning call
//   empties a set the answer is "no" at once.
#include "launch.hpp"
#include "scan.hpp"

namespace gd {

__device__ __forceinline__ uint32_t uf_find(uint32_t* parent, uint32_t x) {
    for (;;) {
        const uint32_t p = load_acq(&parent[x]);
        if (p == x) return x;
        const uint32_t gp = load_acq(&parent[p]);
        if (gp != p) store_rel(&parent[x], gp);
        x = gp;
    }
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

// A run of points: coordinate k of position i at crd[k * kstride + (base + i) * pstride].
struct PointSet {
    const int32_t* crd;
    int64_t kstride;
    int64_t pstride;
    uint32_t base;        // first position of the set
    uint32_t m;           // size
    uint64_t* alive;      // LDS bitmap, ceil(m / 64) words
    uint32_t words;
};

template <int D>
__device__ __forceinline__ void load_point(const PointSet& s, uint32_t pos, int32_t (&x)[D]) {
    const int32_t* p = s.crd + (int64_t)(s.base + pos) * s.pstride;
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = p[(int64_t)k * s.kstride];
}

constexpr uint32_t kUnroll = 4;  // words of a set whose loads are issued together

// Loads the point of this lane in word w (position clamped into the set so
// the address is always valid; callers ignore lanes whose bit is clear).
template <int D>
__device__ __forceinline__ void load_lane_point(const PointSet& s, uint32_t w, int32_t (&x)[D]) {
    uint32_t pos = w * kWave + lane_id();
    pos = pos < s.m ? pos : s.m - 1;
    load_point<D>(s, pos, x);
}

// argmin over live y of D(p, y): returns (D << 32 | position)
template <int D>
__device__ __forceinline__ uint64_t nearest(const PointSet& s, const int32_t (&p)[D], unsigned long long& ndist) {
    const int lane = lane_id();
    uint64_t best = ~0ull;
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
                best = cand < best ? cand : best;
            }
        }
    }
    return wave_min_u64(best);
}

__device__ __forceinline__ double wave_min_f64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(v, o);
        v = t < v ? t : v;
    }
    return v;
}

// Algorithm 4: remove from `a` the points that cannot be within eps of any
// live point of `b`, given anchor p in a and q = argmin_{y in b} D(p, y) with
// D(p, q) = dpq > T.  Returns whether `a` keeps any point.
template <int D>
__device__ __forceinline__ bool pruning(const PointSet& a, const PointSet& b, const int32_t (&p)[D],
                                        const int32_t (&q)[D], uint32_t dpq, uint32_t T, double eps,
                                        unsigned long long& ndist) {
    const int lane = lane_id();
    int32_t pq[D];
#pragma unroll
    for (int k = 0; k < D; ++k) pq[k] = q[k] - p[k];
    const double a2 = (double)dpq;
    const double na = sqrt(a2);
    // lambda over the live points of b
    double cmin = 2.0;
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
            uint32_t b2 = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                py[k] = yy[u][k] - p[k];
                dot += (int64_t)pq[k] * py[k];
                b2 += sq24(yy[u][k], p[k]);
            }
            const double dotd = (double)dot;
            const double h2 = (double)(b2 - T);  // b^2 - eps^2 > 0 since b^2 >= dpq > T
            if (dot < 0 && dotd * dotd >= a2 * h2 * (1.0 - 1e-9)) {
                off = true;  // lambda_y >= pi (or too close to tell)
            } else {
                double cross = 0.0;  // |pq|^2 |py|^2 - (pq.py)^2 as a sum of squared 2x2 minors
#pragma unroll
                for (int k = 0; k < D; ++k)
#pragma unroll
                    for (int l = k + 1; l < D; ++l) {
                        const double mnr = (double)((int64_t)pq[k] * py[l] - (int64_t)pq[l] * py[k]);
                        cross += mnr * mnr;
                    }
                const double c = (dotd * sqrt(h2) - eps * sqrt(cross)) / (na * (double)b2);
                cmin = c < cmin ? c : cmin;
            }
        }
    }
    off = ballot(off) != 0;
    cmin = wave_min_f64(cmin);
    const double thr = cmin - 1e-10;
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
                uint32_t ax = 0;
                int64_t dotx = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    ax += sq24(xx[u][k], p[k]);
                    dotx += (int64_t)pq[k] * (xx[u][k] - p[k]);
                }
                const int64_t s = (int64_t)dpq - (int64_t)T - (int64_t)ax;
                const bool tri = s > 0 && (uint64_t)4 * (uint64_t)T * (uint64_t)ax < (uint64_t)s * (uint64_t)s;
                keep = !tri;
                if (keep && !off && ax > 0) {
                    const double cth = (double)dotx / (na * sqrt((double)ax));
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

// Algorithm 5.  Returns 1 (yes), 0 (no) or -1 (iteration bound exceeded).
template <int D>
__device__ int fast_merging(PointSet si, PointSet sj, uint32_t start, uint32_t T, double eps,
                            unsigned long long& ndist, uint32_t& iters) {
    init_alive<D>(si);
    init_alive<D>(sj);
    wave_sync();
    uint32_t p = start;
    const uint32_t bound = si.m + sj.m + 2;
    for (iters = 1;; ++iters) {
        if (iters > bound) return -1;
        int32_t P[D];
        load_point<D>(si, p, P);
        const uint64_t bq = nearest<D>(sj, P, ndist);
        const uint32_t dq = (uint32_t)(bq >> 32), q = (uint32_t)bq;
        if (dq <= T) return 1;
        int32_t Q[D];
        load_point<D>(sj, q, Q);
        if (!pruning<D>(si, sj, P, Q, dq, T, eps, ndist)) return 0;
        const uint64_t bp = nearest<D>(si, Q, ndist);
        const uint32_t dp = (uint32_t)(bp >> 32);
        p = (uint32_t)bp;
        if (dp <= T) return 1;
        load_point<D>(si, p, P);
        if (!pruning<D>(sj, si, Q, P, dp, T, eps, ndist)) return 0;
    }
}

constexpr uint32_t kSmallSet = kTinyCore;

__device__ __forceinline__ void flush_stats(MergeStats* stats, int64_t r, unsigned long long pairs,
                                            unsigned long long skip, unsigned long long test,
                                            unsigned long long yes, unsigned long long iter,
                                            unsigned long long max_it, unsigned long long dist,
                                            unsigned long long pts) {
    // counters are spread over kStatSlots copies (summed on the host) so
    // that same-address atomics do not serialise the kernel
    MergeStats* sl = stats + ((uint64_t)r & (kStatSlots - 1));
    atomicAdd(&sl->pairs, pairs);
    atomicAdd(&sl->skipped, skip);
    atomicAdd(&sl->tests, test);
    atomicAdd(&sl->yes, yes);
    atomicAdd(&sl->iters, iter);
    atomicAdd(&sl->dists, dist);
    atomicMax(&sl->max_iters, max_it);
    atomicAdd(&sl->set_points, pts);
}

// Pairs of tiny core sets (both at most kSmallSet points).  One wave per tiny
// core grid g_i; every lane takes one neighbouring tiny core grid g_j that
// comes later in the visiting order and decides the pair by evaluating its
// |s_i| x |s_j| distances directly: the answer FastMerging gives (Theorem
// 2), without its wave-level iteration.  Only pairs that answer yes touch the
// union-find.  s_i lives in scalar registers.
template <int D>
__global__ __launch_bounds__(kBlock) void merge_small_kernel(GridView gv, CoreOut co, const uint64_t* __restrict__ nei_off,
                                                             const uint32_t* __restrict__ nei,
                                                             const uint32_t* __restrict__ ldf,
                                                             const uint32_t* __restrict__ rank, int64_t r0, int64_t r1,
                                                             uint32_t* parent, MergeStats* stats) {
    const int lane = lane_id();
    const int64_t r = r0 + (int64_t)blockIdx.x * kWavesPerBlock + wave_id();
    if (r >= r1) return;
    const uint32_t T = (uint32_t)gv.T;
    const uint32_t ci = ldf[r];
    const uint32_t bi = co.core_start[ci];
    const uint32_t mi = co.core_start[ci + 1] - bi;
    if (mi > kSmallSet) return;
    const int P = co.cstride;
    int32_t pi[kSmallSet][D];
#pragma unroll
    for (int a = 0; a < (int)kSmallSet; ++a)
#pragma unroll
        for (int k = 0; k < D; ++k)
            pi[a][k] = uniform((uint32_t)a < mi ? co.ccrd[(int64_t)(bi + a) * P + k] : 0);
    unsigned long long n_pairs = 0, n_yes = 0, n_dist = 0, n_pts = 0;
    const uint64_t e0 = nei_off[ci], e1 = nei_off[ci + 1];
    for (uint64_t e = e0; e < e1; e += kWave) {
        const uint64_t idx = e + lane;
        bool cand = false;
        uint32_t cj = 0, bj = 0, mj = 0;
        if (idx < e1) {
            cj = nei[idx];
            const uint32_t rj = rank[cj];
            if (rj != kNone && rj > (uint32_t)r) {
                bj = co.core_start[cj];
                mj = co.core_start[cj + 1] - bj;
                cand = mj <= kSmallSet;
            }
        }
        bool yes = false;
        if (cand) {
            for (uint32_t b = 0; b < mj && !yes; ++b) {
                int32_t y[D];
#pragma unroll
                for (int k = 0; k < D; ++k) y[k] = co.ccrd[(int64_t)(bj + b) * P + k];
#pragma unroll
                for (int a = 0; a < (int)kSmallSet; ++a) {
                    if ((uint32_t)a < mi) {
                        uint32_t dd = 0;
#pragma unroll
                        for (int k = 0; k < D; ++k) dd += sq24(y[k], pi[a][k]);
                        yes |= dd <= T;
                    }
                }
            }
            if (yes && uf_find(parent, ci) != uf_find(parent, cj)) uf_union(parent, ci, cj);
        }
        if (stats) {
            const unsigned long long np = (unsigned long long)popc64(ballot(cand));
            const unsigned long long sj = (unsigned long long)wave_sum(cand ? mj : 0u);
            n_pairs += np;
            n_yes += (unsigned long long)popc64(ballot(yes));
            n_dist += (unsigned long long)mi * sj;
            n_pts += np * mi + sj;
        }
    }
    // each one-lane test counts as one FastMerging iteration
    if (stats && lane == 0)
        flush_stats(stats, r, n_pairs, 0, n_pairs, n_yes, n_pairs, n_pairs ? 1 : 0, n_dist, n_pts);
}

// Every other pair: one wave per core grid g_i with more than kSmallSet core
// points, in the visiting order.  It takes the neighbouring core grids g_j
// that are tiny (those pairs are tested from this side) or that come later
// in the order, drops the ones already in g_i's set (each lane resolves its
// candidate's root in the same round) and runs FastMerging on the wave for
// each remaining pair, unioning on yes.
template <int D>
__global__ __launch_bounds__(kBlock) void merge_big_kernel(GridView gv, CoreOut co, const uint64_t* __restrict__ nei_off,
                                                           const uint32_t* __restrict__ nei,
                                                           const uint32_t* __restrict__ ldf,
                                                           const uint32_t* __restrict__ rank, int64_t r0, int64_t r1,
                                                           uint32_t words, double eps, uint32_t* parent,
                                                           MergeStats* stats, uint32_t* err) {
    extern __shared__ uint64_t smem[];
    const int lane = lane_id();
    const int wpb = (int)(blockDim.x / kWave);
    const int w = wave_id();
    const int64_t r = r0 + (int64_t)blockIdx.x * wpb + w;
    if (r >= r1) return;
    const uint32_t T = (uint32_t)gv.T;
    const uint32_t ci = ldf[r];
    const int64_t P = co.cstride;
    PointSet si{co.ccrd, 1, P, co.core_start[ci], co.core_start[ci + 1] - co.core_start[ci],
                smem + (int64_t)w * 2 * words, 0};
    if (si.m <= kSmallSet) return;
    si.words = (si.m + kWave - 1) / kWave;
    PointSet sj{co.ccrd, 1, P, 0, 0, smem + (int64_t)w * 2 * words + words, 0};
    unsigned long long n_pairs = 0, n_skip = 0, n_test = 0, n_yes = 0, n_iter = 0, n_dist = 0, max_it = 0, n_pts = 0;
    const uint64_t e0 = nei_off[ci], e1 = nei_off[ci + 1];
    uint32_t ri = uf_find(parent, ci);
    for (uint64_t e = e0; e < e1; e += kWave) {
        const uint64_t idx = e + lane;
        uint32_t cj = 0, bj = 0, mj = 0;
        bool cand = false;
        if (idx < e1) {
            cj = nei[idx];
            const uint32_t rj = rank[cj];
            if (rj != kNone) {
                bj = co.core_start[cj];
                mj = co.core_start[cj + 1] - bj;
                cand = mj <= kSmallSet || rj > (uint32_t)r;
            }
        }
        const bool pend_l = cand && uf_find(parent, cj) != ri;
        const uint64_t cands = ballot(cand);
        uint64_t pend = ballot(pend_l);
        n_pairs += (unsigned long long)popc64(cands);
        n_skip += (unsigned long long)(popc64(cands) - popc64(pend));
        while (pend) {
            const int l = ffs64(pend);
            pend &= pend - 1ull;
            const uint32_t j = readlane(cj, l);
            sj.base = readlane(bj, l);
            sj.m = readlane(mj, l);
            sj.words = (sj.m + kWave - 1) / kWave;
            uint32_t it = 0;
            const int yes = fast_merging<D>(si, sj, 0u, T, eps, n_dist, it);
            ++n_test;
            n_pts += si.m + sj.m;
            n_iter += it;
            max_it = it > max_it ? it : max_it;
            if (yes < 0) {
                if (lane == 0) atomicOr(err, kErrMergeRunaway);
                continue;
            }
            if (yes) {
                ++n_yes;
                if (lane == 0) uf_union(parent, ci, j);
                ri = uf_find(parent, ci);
                if (pend) {
                    // the union may have joined g_i to other pending grids' sets
                    const bool still = ((pend >> lane) & 1ull) && uf_find(parent, cj) != ri;
                    const uint64_t np = ballot(still);
                    n_skip += (unsigned long long)(popc64(pend) - popc64(np));
                    pend = np;
                }
            }
        }
    }
    if (stats && lane == 0) flush_stats(stats, r, n_pairs, n_skip, n_test, n_yes, n_iter, max_it, n_dist, n_pts);
}

hipError_t launch_merge(const GridView& g, const CoreOut& c, const uint64_t* nei_off, const uint32_t* nei,
                        const uint32_t* ldf_list, const uint32_t* rank, int64_t ncc, int64_t n_small, int64_t max_core,
                        int64_t eps, uint32_t* parent, MergeStats* stats, uint32_t* err, hipStream_t st) {
    if (ncc == 0) return hipSuccess;
    // n_small >= 0: the visiting order puts the n_small tiny core grids first
    // (ascending core count); otherwise every wave checks its grid's size.
    const int64_t s1 = n_small >= 0 ? n_small : ncc;
    const int64_t b0 = n_small >= 0 ? n_small : 0;
    if (s1 > 0) {
        const unsigned blocks = (unsigned)((s1 + kWavesPerBlock - 1) / kWavesPerBlock);
        GD_DISPATCH_D(g.d, (merge_small_kernel<D><<<dim3(blocks), dim3(kBlock), 0, st>>>(
                               g, c, nei_off, nei, ldf_list, rank, 0, s1, parent, stats)));
    }
    if (ncc - b0 <= 0 || max_core <= (int64_t)kSmallSet) return hipGetLastError();
    const uint32_t words = (uint32_t)((max_core + kWave - 1) / kWave);
    int wpb = kWavesPerBlock;
    size_t lds = (size_t)wpb * 2 * words * sizeof(uint64_t);
    if (lds > 65536) {
        wpb = 1;
        lds = (size_t)2 * words * sizeof(uint64_t);
    }
    if (lds > 65536) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((ncc - b0 + wpb - 1) / wpb);
    GD_DISPATCH_D(g.d, (merge_big_kernel<D><<<dim3(blocks), dim3(wpb * kWave), lds, st>>>(
                           g, c, nei_off, nei, ldf_list, rank, b0, ncc, words, (double)eps, parent, stats, err)));
    return hipGetLastError();
}

// FastMerging on caller-given pairs of point runs (one wave per pair).
template <int D>
__global__ __launch_bounds__(kBlock) void merge_pairs_kernel(const int32_t* __restrict__ pts, int64_t m,
                                                             const uint32_t* __restrict__ pairs, int64_t npairs,
                                                             uint32_t T, double eps, uint32_t words,
                                                             uint8_t* __restrict__ answers, uint32_t* iterations) {
    extern __shared__ uint64_t smem[];
    const int wpb = (int)(blockDim.x / kWave);
    const int w = wave_id();
    const int64_t r = (int64_t)blockIdx.x * wpb + w;
    if (r >= npairs) return;
    PointSet a{pts, m, 1, pairs[4 * r], pairs[4 * r + 1], smem + (int64_t)w * 2 * words, 0};
    PointSet b{pts, m, 1, pairs[4 * r + 2], pairs[4 * r + 3], smem + (int64_t)w * 2 * words + words, 0};
    a.words = (a.m + kWave - 1) / kWave;
    b.words = (b.m + kWave - 1) / kWave;
    unsigned long long nd = 0;
    uint32_t it = 0;
    const int yes = fast_merging<D>(a, b, 0u, T, eps, nd, it);
    if (lane_id() == 0) {
        answers[r] = yes < 0 ? 2 : (uint8_t)yes;
        if (iterations) iterations[r] = it;
    }
}

hipError_t launch_merge_pairs(const int32_t* pts, int64_t m, int d, const uint32_t* pairs, int64_t npairs,
                              int64_t eps, uint32_t max_count, uint8_t* answers, uint32_t* iterations,
                              hipStream_t st) {
    if (npairs == 0) return hipSuccess;
    const uint32_t words = (max_count + kWave - 1) / kWave;
    int wpb = kWavesPerBlock;
    size_t lds = (size_t)wpb * 2 * words * sizeof(uint64_t);
    if (lds > 65536) {
        wpb = 1;
        lds = (size_t)2 * words * sizeof(uint64_t);
    }
    if (lds > 65536) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((npairs + wpb - 1) / wpb);
    GD_DISPATCH_D(d, (merge_pairs_kernel<D><<<dim3(blocks), dim3(wpb * kWave), lds, st>>>(
                         pts, m, pairs, npairs, (uint32_t)(eps * eps), (double)eps, words, answers, iterations)));
    return hipGetLastError();
}

__global__ __launch_bounds__(kBlock) void root_min_kernel(int64_t ncell, const uint32_t* core_start,
                                                          const uint32_t* cell_min_core, uint32_t* parent,
                                                          uint32_t* root_min) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncell || core_start[c + 1] == core_start[c]) return;
    atomicMin(&root_min[uf_find(parent, (uint32_t)c)], cell_min_core[c]);
}

__global__ __launch_bounds__(kBlock) void cell_label_kernel(int64_t ncell, const uint32_t* core_start,
                                                            uint32_t* parent, const uint32_t* root_min,
                                                            int32_t* cell_label) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= ncell) return;
    cell_label[c] = core_start[c + 1] == core_start[c] ? -1 : (int32_t)root_min[uf_find(parent, (uint32_t)c)];
}

hipError_t launch_labels(const GridView& g, const CoreOut& c, uint32_t* parent, uint32_t* root_min,
                         int32_t* cell_label, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    hipError_t e = fill<uint32_t>(root_min, g.ncell, kNone, st);
    if (e != hipSuccess) return e;
    root_min_kernel<<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(g.ncell, c.core_start, c.cell_min_core, parent,
                                                                      root_min);
    cell_label_kernel<<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(g.ncell, c.core_start, parent, root_min,
                                                                        cell_label);
    return hipGetLastError();
}

}  // namespace gd
