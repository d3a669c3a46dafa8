// Merging core grids (Section 4.3) with union-find over core grids visited
// in ascending core-count order (the LDF variant of Section 5.2); the
// FastMerging test itself is in fastmerge.hpp.
#include <algorithm>
#include <type_traits>

#include "fastmerge.hpp"
#include "fastmerge_block.hpp"
#include "launch.hpp"
#include "learned.hpp"
#include "scan.hpp"

namespace gd {

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

// Pairs of tiny core sets (both at most kSmallSet points).  S lanes per tiny
// core grid g_i (a wave serves 64 / S grids: with short lists, as with
// millions of sparse grids, most of a wave per grid would idle); every lane
// takes one neighbouring tiny core grid g_j with a larger grid index (each
// pair once, from its lower grid: the tiny core grids are all visited by
// this one launch, so their order among themselves is immaterial, and half
// of the list needs no load at all) and decides the pair by evaluating its
// |s_i| x |s_j| distances directly: the answer FastMerging gives
// (Theorem 2), without its wave-level iteration.  Each lane first resolves
// its candidate's root and skips the pair when both grids are already in
// one set; a yes joins the two roots.  With S = 64, s_i lives in scalar
// registers.
template <int D, bool kWide, int S>
__global__ __launch_bounds__(kBlock) void merge_small_kernel(GridView gv, CoreOut co, const uint64_t* __restrict__ nei_off,
                                                             const uint32_t* __restrict__ nei,
                                                             const uint2* __restrict__ nei_up,
                                                             const uint32_t* __restrict__ ldf,
                                                             const uint4* __restrict__ rank, int64_t r0, int64_t r1,
                                                             const uint32_t* split, uint32_t* parent,
                                                             MergeStats* stats) {
    constexpr int G = kWave / S;  // grids per wave
    const int lane = lane_id();
    const int grp = lane / S, sub = lane % S;
    const uint64_t gmask = (S == kWave ? ~0ull : ((1ull << S) - 1ull)) << (grp * S);
    const int64_t r = r0 + (block_id() * kWavesPerBlock + wave_id()) * G + grp;
    // lanes of a group without a tiny core grid take an empty list, so that
    // every lane reaches the closing reductions
    bool live = r < r1 && r < (int64_t)co.counts[1] && !(split && r >= (int64_t)*split);
    const uint32_t ci = live ? ldf[r] : 0u;
    // every load that depends on ci alone is issued before the first use
    // the merge's "yes" bound: eps^2, or (eps + delta)^2 when approximate
    const typename Dist<kWide>::T T = inst_Tm<kWide>(cell_inst(gv, ci));
    const uint4 own = live ? rank[ci] : make_uint4(0u, 0u, 0u, 0u);
    uint64_t e0 = live ? nei_off[ci] : 0, e1 = live ? nei_off[ci + 1] : 0;
    if (nei_up && live) {
        // lists in walk order: only the range of larger-index neighbours
        const uint2 up = nei_up[ci];
        e1 = e0 + up.y;
        e0 += up.x;
    }
    const uint32_t pci = load_acq(&parent[ci]);
    const uint32_t bi = own.y;
    const uint32_t mi = own.z;
    if (mi > kSmallSet) live = false;
    if (!live) e0 = e1 = 0;
    int32_t pi[kSmallSet][D];
#pragma unroll
    for (int a = 0; a < (int)kSmallSet; ++a) {
        int32_t t[D];
        load_row<D>(co.ccrd, (uint32_t)a < mi ? bi + a : bi, t);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int32_t v = (uint32_t)a < mi ? t[k] : 0;
            if constexpr (S == kWave)
                pi[a][k] = uniform(v);
            else
                pi[a][k] = v;
        }
    }
    unsigned long long n_pairs = 0, n_skip = 0, n_yes = 0, n_dist = 0, n_pts = 0;
    uint32_t ri = live ? uf_find_at(parent, ci, pci) : 0u;  // root hint of g_i's set
    // each round takes two list entries per lane (four with a wave per
    // grid), whose loads are issued together: the rounds are chains of
    // dependent loads, so fewer rounds cost less time (with a wave per grid
    // the lists are long: cfg2's merge 40.6 -> 38.6 ms from two to four)
    constexpr int U = S == kWave ? 4 : 2;
    for (uint64_t e = e0; e < e1; e += U * S) {
        bool cand[U];
        uint32_t cj[U], bj[U], mj[U], pj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t idx = e + (uint64_t)u * S + sub;
            cand[u] = false;
            cj[u] = bj[u] = mj[u] = pj[u] = 0;
            if (idx < e1) cj[u] = nei[idx];
        }
        // the root of each candidate first: a pair already in one set (most
        // of them once the merge is under way) needs no 16-byte record load
        // (it is still read when counting, so that the counts keep their
        // meaning); the root found is the hint for the union
        uint32_t root_j[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            pj[u] = cj[u] > ci ? load_acq(&parent[cj[u]]) : 0u;
            root_j[u] = cj[u] > ci ? uf_find_at(parent, cj[u], pj[u]) : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (cj[u] > ci && (root_j[u] != ri || stats)) {
                const uint4 rc = rank[cj[u]];
                if (rc.x != kNone) {
                    bj[u] = rc.y;
                    mj[u] = rc.z;
                    cand[u] = mj[u] <= kSmallSet;
                }
            }
        }
        bool any_yes = false;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool test = cand[u] && root_j[u] != ri;
            bool yes = false;
            if (test) {
                // four rows of s_j per round, loaded together (a repeated last
                // row only repeats a distance)
                for (uint32_t b0 = 0; b0 < mj[u] && !yes; b0 += 4) {
                    int32_t y[4][D];
#pragma unroll
                    for (int v = 0; v < 4; ++v) load_row<D>(co.ccrd, bj[u] + min(b0 + v, mj[u] - 1), y[v]);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
#pragma unroll
                        for (int a = 0; a < (int)kSmallSet; ++a) {
                            if ((uint32_t)a < mi) {
                                typename Dist<kWide>::T dd = 0;
#pragma unroll
                                for (int k = 0; k < D; ++k) dd += sqd<kWide>(y[v][k], pi[a][k]);
                                yes |= dd <= T;
                            }
                        }
                    }
                }
                // a stale root only costs this lane's union a second find
                if (yes) uf_union_from(parent, ri, root_j[u]);
            }
            any_yes |= yes;
            if (stats) {
                n_pairs += cand[u] ? 1u : 0u;
                n_skip += cand[u] && !test ? 1u : 0u;
                n_yes += yes ? 1u : 0u;
                n_dist += test ? (unsigned long long)mi * mj[u] : 0ull;
                n_pts += test ? (unsigned long long)(mi + mj[u]) : 0ull;
            }
        }
        // the unions may have put g_i's set under a smaller root
        if (ballot(any_yes) & gmask) ri = uf_find(parent, ri);
    }
    // each one-lane test counts as one FastMerging iteration
    if (stats) {
        n_pairs = wave_sum(n_pairs);
        n_skip = wave_sum(n_skip);
        n_yes = wave_sum(n_yes);
        n_dist = wave_sum(n_dist);
        n_pts = wave_sum(n_pts);
        if (lane == 0) {
            const unsigned long long nt = n_pairs - n_skip;
            flush_stats(stats, r, n_pairs, n_skip, nt, n_yes, nt, nt ? 1 : 0, n_dist, n_pts);
        }
    }
}

// Queues the pairs (g_i, g_j) of the lanes in `lanes` (each lane holds its
// g_j) for merge_huge_kernel, with one append for the wave.
__device__ __noinline__ void defer_pairs(const HugeQueue& q, uint64_t lanes, uint32_t ci, uint32_t cj, Header* hdr) {
    const int lane = lane_id();
    uint32_t base = 0;
    if (lane == 0) base = q.pairs ? atomicAdd(q.count, (uint32_t)popc64(lanes)) : q.cap;
    base = readlane(base, 0);
    if ((lanes >> lane) & 1ull) {
        const uint32_t k = base + (uint32_t)popc64(lanes & lanemask_lt());
        if (k < q.cap)
            q.pairs[k] = make_uint2(ci, cj);
        else
            atomicOr(&hdr->err, kErrCoreCap);
    }
}

// Every other pair: one wave per core grid g_i with more than kSmallSet core
// points, in the visiting order.  It takes the neighbouring core grids g_j
// that are tiny (those pairs are tested from this side) or that come later
// in the order, drops the ones already in g_i's set (each lane resolves its
// candidate's root in the same round) and runs FastMerging on the wave for
// each remaining pair, unioning on yes.
// Learned proposal (kLearned): the scorer orders each chunk's remaining
// pairs by their merge logit (likely merges first, so the unions they make
// let later pairs be skipped) and picks the starting side and point; the
// FastMerging answer is the same whatever it picks.
struct Proposal {
    const __half* weights;     // FP16 parameter vector
    const CellSummary* sum;    // per core grid
};

__device__ __forceinline__ uint32_t orderable(float z) {
    const uint32_t u = __float_as_uint(z);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// The kernel is bound by the latency of union-find and FastMerging steps:
// six waves per SIMD (at most 85 registers) hide more of it than wider
// unrolling inside a wave.  The scorer's fragments, and rows of d >= 5, do
// not fit in that budget (they would spill to scratch), so those variants
// run four.
template <int D, bool kLearned, bool kWide>
__global__ __launch_bounds__(kBlock, (kLearned || D >= 5) ? 4 : 6) void merge_big_kernel(GridView gv, CoreOut co, const uint64_t* __restrict__ nei_off,
                                                           const uint32_t* __restrict__ nei,
                                                           const uint32_t* __restrict__ ldf,
                                                           const uint4* __restrict__ rank, int64_t r0, int64_t r1,
                                                           const uint32_t* split, uint32_t words, HugeQueue huge,
                                                           uint32_t* parent, MergeStats* stats, Proposal prop) {
    extern __shared__ uint64_t smem[];
    using Weights = typename std::conditional<kLearned, MlpMfma, float>::type;
    using Scratch = typename std::conditional<kLearned, MlpMfmaScratch, float>::type;
    __shared__ Weights W[1];
    __shared__ Scratch S[kLearned ? kWavesPerBlock : 1];
    __shared__ float2 zb[kLearned ? kWavesPerBlock : 1][kLearned ? kWave : 1];
    if constexpr (kLearned) {
        mlp_mfma_load(W[0], prop.weights);
        __syncthreads();
    }
    const int lane = lane_id();
    const int wpb = (int)(blockDim.x / kWave);
    const int w = wave_id();
    // with a device split the big core sets start right after the tiny ones
    const int64_t r = (split ? (int64_t)*split : r0) + block_id() * wpb + w;
    if (r >= r1 || r >= (int64_t)co.counts[1]) return;
    const uint32_t ci = ldf[r];
    // every load that depends on ci alone is issued before the first use
    const Inst& I = cell_inst(gv, ci);
    const uint4 own = rank[ci];
    const uint64_t e0 = nei_off[ci], e1 = nei_off[ci + 1];
    const uint32_t pci = load_acq(&parent[ci]);
    const typename Dist<kWide>::T T = inst_T<kWide>(I), Tm = inst_Tm<kWide>(I);
    const double eps = (double)I.eps;
    PointSet si{co.ccrd, own.y, own.z, smem + (int64_t)w * 2 * words, 0};
    if (si.m <= kSmallSet) return;
    // larger than the LDS bitmaps this launch was given (or heavy, with a
    // queue): every pair is queued
    const bool si_huge = si.m > 64u * words;
    const bool si_heavy = huge.pairs && si.m >= (uint32_t)kHeavyCore;
    if (si_huge && !huge.pairs) {
        if (lane == 0) atomicOr(&gv.b.hdr->err, kErrCoreCap);
        return;
    }
    si.words = (si.m + kWave - 1) / kWave;
    // the plain tests all start from s_i's first point: loaded once
    int32_t p0[D];
    load_point<D>(si, 0u, p0);
    PointSet sj{co.ccrd, 0, 0, smem + (int64_t)w * 2 * words + words, 0};
    unsigned long long n_pairs = 0, n_skip = 0, n_test = 0, n_yes = 0, n_iter = 0, n_dist = 0, max_it = 0, n_pts = 0;
    uint32_t ri = uf_find_at(parent, ci, pci);
    for (uint64_t e = e0; e < e1; e += kWave) {
        const uint64_t idx = e + lane;
        uint32_t cj = 0, bj = 0, mj = 0, pj = 0;
        bool cand = false;
        if (idx < e1) {
            cj = nei[idx];
            // the parent link loads beside the record (every grid has one)
            pj = load_acq(&parent[cj]);
            const uint4 rc = rank[cj];
            const uint32_t rj = rc.x;
            if (rj != kNone) {
                bj = rc.y;
                mj = rc.z;
                cand = mj <= kSmallSet || rj > (uint32_t)r;
            }
        }
        // root of each candidate's set, kept as the hint for a union
        uint32_t root_j = cand ? uf_find_at(parent, cj, pj) : 0u;
        const bool pend_l = cand && root_j != ri;
        const uint64_t cands = ballot(cand);
        uint64_t pend = ballot(pend_l);
        n_pairs += (unsigned long long)popc64(cands);
        n_skip += (unsigned long long)(popc64(cands) - popc64(pend));
        // pairs with a core set beyond the LDS bitmaps, or (eager runs) with
        // a heavy one, go to the queue
        const uint64_t over =
            ballot(pend_l && (si_huge || si_heavy || mj > 64u * words || (huge.pairs && mj >= (uint32_t)kHeavyCore)));
        if (over) {
            defer_pairs(huge, over, ci, cj, gv.b.hdr);
            pend &= ~over;
        }
        float my_z0 = 0.f, my_z1 = 0.f;
        uint32_t my_ra = 0, my_rb = 0;
        if constexpr (kLearned) {
            // score every pending pair: features per lane, the scorer on the
            // matrix cores 16 pairs at a time
            const bool pl = ((pend >> lane) & 1ull) && mj <= 64u * words;
            const uint64_t pm = ballot(pl);
            const uint32_t rk = (uint32_t)popc64(pm & lanemask_lt());
            const int np = popc64(pm);
            float f[kFeat];
            uint32_t ra = 0, rb = 0;
            if (pl) pair_setup<D>(gv, co, prop.sum, ci, cj, eps, f, ra, rb);
            my_ra = ra;
            my_rb = rb;
            for (int b0 = 0; b0 < np; b0 += 16) {
                if (pl && rk >= (uint32_t)b0 && rk < (uint32_t)b0 + 16u) {
#pragma unroll
                    for (int k = 0; k < kFeat; ++k) S[w].feat[rk - b0][k] = (_Float16)f[k];
                }
                wave_sync();
                float z0[4], z1[4];
                mlp_forward_mfma(W[0], S[w], z0, z1);
                if ((lane & 15) == 0) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) zb[w][b0 + 4 * (lane >> 4) + j] = make_float2(z0[j], z1[j]);
                }
                wave_sync();
            }
            if (pl) {
                my_z0 = zb[w][rk].x;
                my_z1 = zb[w][rk].y;
            }
            wave_sync();
        }
        while (pend) {
            int l;
            if constexpr (kLearned) {
                // the remaining pair with the largest merge logit (ties: lowest
                // lane); every pending lane's key is >= 64 > 0, the others' key
                const uint64_t key = ((pend >> lane) & 1ull)
                                         ? (((uint64_t)orderable(my_z0) << 7) | 64ull | (uint64_t)(kWave - 1 - lane))
                                         : 0ull;
                const uint64_t best = ~wave_min_u64(~key);
                l = kWave - 1 - (int)(best & 63ull);
            } else {
                l = ffs64(pend);
            }
            pend &= ~(1ull << l);
            sj.base = readlane(bj, l);
            sj.m = readlane(mj, l);
            sj.words = (sj.m + kWave - 1) / kWave;
            uint32_t it = 0;
            int yes;
            if constexpr (kLearned) {
                if (__shfl(my_z1, l) > 0.f)
                    yes = fast_merging<D, kWide>(sj, si, readlane(my_rb, l), T, Tm, eps, n_dist, it);
                else
                    yes = fast_merging<D, kWide>(si, sj, readlane(my_ra, l), T, Tm, eps, n_dist, it);
            } else {
                // start in the larger set, so that the first nearest-point
                // search (on a yes the only one) runs over the smaller set
                const bool swap = sj.m > si.m;
                int32_t ps[D];
                if (swap) load_point<D>(sj, 0u, ps);
#pragma unroll
                for (int k = 0; k < D; ++k) ps[k] = swap ? ps[k] : p0[k];
                yes = fast_merging_from<D, kWide>(swap ? sj : si, swap ? si : sj, ps, T, Tm, eps, n_dist, it);
            }
            ++n_test;
            n_pts += si.m + sj.m;
            n_iter += it;
            max_it = it > max_it ? it : max_it;
            if (yes < 0) {
                if (lane == 0) atomicOr(&gv.b.hdr->err, kErrMergeRunaway);
                continue;
            }
            if (yes) {
                ++n_yes;
                const uint32_t rl = readlane(root_j, l);
                uint32_t root = 0;
                if (lane == 0) root = uf_union_from(parent, ri, rl);
                ri = readlane(root, 0);
                if (pend) {
                    // the union may have joined g_i to other pending grids' sets
                    const bool pl = (pend >> lane) & 1ull;
                    if (pl) root_j = uf_find(parent, root_j);
                    const bool still = pl && root_j != ri;
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
                        const uint2* nei_up,
                        const uint32_t* ldf_list, const uint4* rank, int64_t ncc, int64_t n_small, int64_t max_core,
                        int waves, int small_lanes, bool tiny_done, const HugeQueue& huge, bool wide,
                        uint32_t* parent, MergeStats* stats, const __half* proposal, const CellSummary* sum,
                        hipStream_t st) {
    const Proposal prop{proposal, sum};
    if (ncc == 0) return hipSuccess;
    // n_small >= 0: the visiting order puts the n_small tiny core grids first
    // (ascending core count).  n_small == -2: the same order, but the count
    // is only known on the device (split); both kernels get grids for all
    // ncc ranks and leave the other kernel's ranks alone.  n_small == -1: no
    // such order; every wave checks its grid's size.
    const uint32_t* split = n_small == -2 ? &c.counts[4] : nullptr;
    const int64_t s1 = n_small >= 0 ? n_small : ncc;
    const int64_t b0 = n_small >= 0 ? n_small : 0;
    if (s1 > 0 && !tiny_done) {
        // lanes per tiny grid: 16 (four grids per wave) or 64
        const int S = small_lanes == 16 ? 16 : kWave;
        const int64_t per_block = (int64_t)kWavesPerBlock * (kWave / S);
        const dim3 blocks = grid_of((s1 + per_block - 1) / per_block), threads(kBlock);
        if (wide && S == 16)
            GD_DISPATCH_D(g.D, (merge_small_kernel<D, true, 16><<<blocks, threads, 0, st>>>(
                                   g, c, nei_off, nei, nei_up, ldf_list, rank, 0, s1, split, parent, stats)));
        else if (wide)
            GD_DISPATCH_D(g.D, (merge_small_kernel<D, true, kWave><<<blocks, threads, 0, st>>>(
                                   g, c, nei_off, nei, nei_up, ldf_list, rank, 0, s1, split, parent, stats)));
        else if (S == 16)
            GD_DISPATCH_D(g.D, (merge_small_kernel<D, false, 16><<<blocks, threads, 0, st>>>(
                                   g, c, nei_off, nei, nei_up, ldf_list, rank, 0, s1, split, parent, stats)));
        else
            GD_DISPATCH_D(g.D, (merge_small_kernel<D, false, kWave><<<blocks, threads, 0, st>>>(
                                   g, c, nei_off, nei, nei_up, ldf_list, rank, 0, s1, split, parent, stats)));
    }
    if (ncc - b0 <= 0 || max_core <= (int64_t)kSmallSet) return hipGetLastError();
    const uint32_t words = (uint32_t)((std::min<int64_t>(max_core, kMaxCoreBits) + kWave - 1) / kWave);
    int wpb = std::max(1, std::min(waves, kWavesPerBlock));
    while (wpb > 1 && (size_t)wpb * 2 * words * sizeof(uint64_t) > 65536) wpb >>= 1;
    const size_t lds = (size_t)wpb * 2 * words * sizeof(uint64_t);
    if (lds > 65536) return hipErrorInvalidValue;
    const dim3 blocks = grid_of((ncc - b0 + wpb - 1) / wpb);
    // the scorer's weights take static LDS beside the bitmaps; if both do not
    // fit, or on the wide path, run without the proposal (the answers are the
    // same)
    const bool learned = prop.weights && !wide &&
                         lds + sizeof(MlpMfma) + kWavesPerBlock * (sizeof(MlpMfmaScratch) + sizeof(float2) * kWave) <=
                             65536;
    if (learned) {
        GD_DISPATCH_D(g.D, (merge_big_kernel<D, true, false><<<blocks, dim3(wpb * kWave), lds, st>>>(
                               g, c, nei_off, nei, ldf_list, rank, b0, ncc, split, words, huge, parent, stats, prop)));
    } else if (wide) {
        GD_DISPATCH_D(g.D, (merge_big_kernel<D, false, true><<<blocks, dim3(wpb * kWave), lds, st>>>(
                               g, c, nei_off, nei, ldf_list, rank, b0, ncc, split, words, huge, parent, stats, prop)));
    } else {
        GD_DISPATCH_D(g.D, (merge_big_kernel<D, false, false><<<blocks, dim3(wpb * kWave), lds, st>>>(
                               g, c, nei_off, nei, ldf_list, rank, b0, ncc, split, words, huge, parent, stats, prop)));
    }
    return hipGetLastError();
}

// ---- The BFS merge order of Algorithm 6 (Section 4.4), for comparison with
// LDF.  Algorithm 6 starts a breadth-first search at an unclassified core
// grid, tests each expanded grid against its unclassified core neighbours
// and claims those FastMerging joins; classified grids are not tested
// again.  Here the searches run level by level, from many seeds at once:
// the seeds of a round are the unclassified core grids with no unclassified
// core neighbour of smaller index (the round's smallest unclassified grid
// is always one, so rounds repeat until every core grid is classified).  A
// neighbour already claimed by another seed's search is tested too when it
// is not yet in the expanding grid's set, and unioned on yes, so searches
// that meet inside one cluster join: the components are those of the
// merge graph whatever the interleaving, as with every order (Theorem 4).

enum : uint32_t { kBfsNew = 0u, kBfsClassified = 1u };

// Seeds of a round: cnt[0] += unclassified core grids, cnt[1] += seeds
// (appended to front).
__global__ __launch_bounds__(kBlock) void bfs_seed_kernel(const uint32_t* ncell, const uint64_t* __restrict__ nei_off,
                                                          const uint32_t* __restrict__ nei,
                                                          const uint32_t* __restrict__ core_cnt,
                                                          uint32_t* __restrict__ state, uint32_t* __restrict__ front,
                                                          uint32_t* cnt) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool open = false, seed = false;
    if (c < (int64_t)*ncell && core_cnt[c] != 0 && state[c] == kBfsNew) {
        open = true;
        seed = true;
        for (uint64_t e = nei_off[c]; e < nei_off[c + 1] && seed; ++e) {
            const uint32_t a = nei[e];
            if (a < (uint32_t)c && core_cnt[a] != 0 && state[a] == kBfsNew) seed = false;
        }
    }
    const uint64_t om = ballot(open), sm = ballot(seed);
    uint32_t base = 0;
    if (lane_id() == 0 && om) {
        atomicAdd(&cnt[0], (uint32_t)popc64(om));
        if (sm) base = atomicAdd(&cnt[1], (uint32_t)popc64(sm));
    }
    base = readlane(base, 0);
    if (seed) {
        front[base + popc64(sm & lanemask_lt())] = (uint32_t)c;
        state[c] = kBfsClassified;
    }
}

// One level: a wave per frontier grid tests its core neighbours that are
// unclassified, or classified outside its set; claimed grids form the next
// frontier (cnt[2]).
template <int D, bool kWide>
__global__ __launch_bounds__(kBlock) void bfs_level_kernel(GridView gv, CoreOut co, const uint64_t* __restrict__ nei_off,
                                                           const uint32_t* __restrict__ nei,
                                                           const uint32_t* __restrict__ front, uint32_t nfront,
                                                           uint32_t* __restrict__ next, uint32_t* cnt, uint32_t words,
                                                           HugeQueue huge, uint32_t* state, uint32_t* parent,
                                                           MergeStats* stats) {
    extern __shared__ uint64_t smem[];
    const int lane = lane_id();
    const int wpb = (int)(blockDim.x / kWave);
    const int w = wave_id();
    const int64_t f = block_id() * wpb + w;
    if (f >= (int64_t)nfront) return;
    const uint32_t ci = front[f];
    const Inst& I = cell_inst(gv, ci);
    const typename Dist<kWide>::T T = inst_T<kWide>(I), Tm = inst_Tm<kWide>(I);
    const double eps = (double)I.eps;
    PointSet si{co.ccrd, co.core_begin[ci], co.core_cnt[ci], smem + (int64_t)w * 2 * words, 0};
    si.words = (si.m + kWave - 1) / kWave;
    const bool si_huge = si.m > 64u * words;  // every pair is queued
    const bool si_heavy = huge.pairs && si.m >= (uint32_t)kHeavyCore;
    if (si_huge && !huge.pairs) {
        if (lane == 0) atomicOr(&gv.b.hdr->err, kErrCoreCap);
        return;
    }
    int32_t p0[D];
    load_point<D>(si, 0u, p0);
    PointSet sj{co.ccrd, 0, 0, smem + (int64_t)w * 2 * words + words, 0};
    unsigned long long n_pairs = 0, n_skip = 0, n_test = 0, n_yes = 0, n_iter = 0, n_dist = 0, max_it = 0, n_pts = 0;
    uint32_t ri = uf_find(parent, ci);
    const uint64_t e0 = nei_off[ci], e1 = nei_off[ci + 1];
    for (uint64_t e = e0; e < e1; e += kWave) {
        const uint64_t idx = e + lane;
        uint32_t cj = 0, mj = 0, sj_state = 0, root_j = 0;
        bool cand = false;
        if (idx < e1) {
            cj = nei[idx];
            mj = co.core_cnt[cj];
            if (mj != 0) {
                cand = true;
                sj_state = load_acq(&state[cj]);
                root_j = uf_find(parent, cj);
            }
        }
        const bool pend_l = cand && (sj_state == kBfsNew || root_j != ri);
        const uint64_t cands = ballot(cand);
        uint64_t pend = ballot(pend_l);
        n_pairs += (unsigned long long)popc64(cands);
        n_skip += (unsigned long long)(popc64(cands) - popc64(pend));
        // pairs with a core set beyond the LDS bitmaps, or (eager runs) with
        // a heavy one, go to the queue
        const uint64_t over =
            ballot(pend_l && (si_huge || si_heavy || mj > 64u * words || (huge.pairs && mj >= (uint32_t)kHeavyCore)));
        if (over) {
            defer_pairs(huge, over, ci, cj, gv.b.hdr);
            pend &= ~over;
        }
        while (pend) {
            const int l = ffs64(pend);
            pend &= pend - 1ull;
            const uint32_t cjl = readlane(cj, l);
            sj.base = co.core_begin[cjl];
            sj.m = readlane(mj, l);
            sj.words = (sj.m + kWave - 1) / kWave;
            // a union since this round's roots were read may have joined them
            if (uf_find(parent, cjl) == uf_find(parent, ri) && load_acq(&state[cjl]) == kBfsClassified) {
                ++n_skip;
                continue;
            }
            uint32_t it = 0;
            // start in the larger set: the first nearest-point search runs over the smaller one
            const bool swap = sj.m > si.m;
            int32_t ps[D];
            if (swap) load_point<D>(sj, 0u, ps);
#pragma unroll
            for (int k = 0; k < D; ++k) ps[k] = swap ? ps[k] : p0[k];
            const int yes = fast_merging_from<D, kWide>(swap ? sj : si, swap ? si : sj, ps, T, Tm, eps, n_dist, it);
            ++n_test;
            n_pts += si.m + sj.m;
            n_iter += it;
            max_it = it > max_it ? it : max_it;
            if (yes < 0) {
                if (lane == 0) atomicOr(&gv.b.hdr->err, kErrMergeRunaway);
                continue;
            }
            if (yes) {
                ++n_yes;
                uint32_t root = 0;
                if (lane == 0) {
                    // claim an unclassified grid for this search; a grid
                    // already classified (by any search) is only unioned
                    if (atomicCAS(&state[cjl], kBfsNew, kBfsClassified) == kBfsNew)
                        next[atomicAdd(&cnt[2], 1u)] = cjl;
                    root = uf_union_from(parent, uf_find(parent, ri), uf_find(parent, cjl));
                }
                ri = readlane(root, 0);
            }
        }
    }
    if (stats && lane == 0) flush_stats(stats, f, n_pairs, n_skip, n_test, n_yes, n_iter, max_it, n_dist, n_pts);
}

hipError_t launch_bfs_seeds(const GridView& g, const CoreOut& c, const uint64_t* nei_off, const uint32_t* nei,
                            uint32_t* state, uint32_t* front, uint32_t* cnt, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    bfs_seed_kernel<<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(g.ncell_dev, nei_off, nei, c.core_cnt, state,
                                                                       front, cnt);
    return hipGetLastError();
}

hipError_t launch_bfs_level(const GridView& g, const CoreOut& c, const uint64_t* nei_off, const uint32_t* nei,
                            const uint32_t* front, uint32_t nfront, uint32_t* next, uint32_t* cnt, int64_t max_core,
                            const HugeQueue& huge, bool wide, uint32_t* state, uint32_t* parent, MergeStats* stats,
                            hipStream_t st) {
    if (nfront == 0) return hipSuccess;
    const uint32_t words =
        (uint32_t)((std::min<int64_t>(std::max<int64_t>(max_core, 1), kMaxCoreBits) + kWave - 1) / kWave);
    int wpb = kWavesPerBlock;
    while (wpb > 1 && (size_t)wpb * 2 * words * sizeof(uint64_t) > 65536) wpb >>= 1;
    const size_t lds = (size_t)wpb * 2 * words * sizeof(uint64_t);
    if (lds > 65536) return hipErrorInvalidValue;
    const dim3 blocks = grid_of(((int64_t)nfront + wpb - 1) / wpb);
    if (wide)
        GD_DISPATCH_D(g.D, (bfs_level_kernel<D, true><<<blocks, dim3(wpb * kWave), lds, st>>>(
                               g, c, nei_off, nei, front, nfront, next, cnt, words, huge, state, parent, stats)));
    else
        GD_DISPATCH_D(g.D, (bfs_level_kernel<D, false><<<blocks, dim3(wpb * kWave), lds, st>>>(
                               g, c, nei_off, nei, front, nfront, next, cnt, words, huge, state, parent, stats)));
    return hipGetLastError();
}

// ---- Core sets larger than the LDS bitmaps.  The merge and BFS kernels
// queue every pair with such a set; the queue is then drained here with the
// two bitmaps of a test in device memory (a slab of 2 * words words per
// wave; each wave owns its slab, and the fences of wave_sync order its
// lanes' accesses as they do in LDS).  The union-find makes the components
// independent of the order of the tests (Theorem 4), so deferring a pair
// changes no answer.

__global__ __launch_bounds__(kBlock) void huge_scan_kernel(const uint32_t* ncell, const uint32_t* __restrict__ core_cnt,
                                                           const uint64_t* __restrict__ nei_off,
                                                           unsigned long long* sum) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c < (int64_t)*ncell && core_cnt[c] >= (uint32_t)kHeavyCore)
        atomicAdd(sum, (unsigned long long)(nei_off[c + 1] - nei_off[c] + 1));
}

// Persistent: workgroup k takes queued pairs k, k + blocks, ... (every
// workgroup leaves once it passes the queue's length, read once at entry),
// and runs FastMerging on each with all of its waves (fastmerge_block.hpp).
template <int D, bool kWide>
__global__ __launch_bounds__(kCoopWaves * kWave) void merge_heavy_kernel(GridView gv, CoreOut co, HugeQueue q,
                                                                         uint64_t* slabs, uint32_t words, int bfs,
                                                                         uint32_t* state, uint32_t* next,
                                                                         uint32_t* cnt, uint32_t* parent,
                                                                         MergeStats* stats) {
    __shared__ BlockScratch<D, kCoopWaves> sh;
    __shared__ uint32_t s_go;
    const int lane = lane_id();
    const bool t0 = threadIdx.x == 0;
    const uint32_t npairs = min(*q.count, q.cap);
    uint64_t* bits = slabs + (int64_t)blockIdx.x * 2 * (int64_t)words;
    unsigned long long n_skip = 0, n_test = 0, n_yes = 0, n_iter = 0, n_dist = 0, max_it = 0, n_pts = 0;
    for (int64_t k = blockIdx.x; k < (int64_t)npairs; k += gridDim.x) {
        const uint2 pr = q.pairs[k];
        const uint32_t ci = pr.x, cj = pr.y;
        uint32_t ri = 0, rj = 0;
        if (t0) {
            ri = uf_find(parent, ci);
            rj = uf_find(parent, cj);
            s_go = (ri == rj && (!bfs || load_acq(&state[cj]) == kBfsClassified)) ? 0u : 1u;
        }
        __syncthreads();
        const bool go = s_go != 0u;
        __syncthreads();
        if (!go) {
            ++n_skip;
            continue;
        }
        const Inst& I = cell_inst(gv, ci);
        PointSet si{co.ccrd, co.core_begin[ci], co.core_cnt[ci], bits, 0};
        PointSet sj{co.ccrd, co.core_begin[cj], co.core_cnt[cj], bits + words, 0};
        si.words = (si.m + kWave - 1) / kWave;
        sj.words = (sj.m + kWave - 1) / kWave;
        if (si.words > words || sj.words > words) {
            if (t0) atomicOr(&gv.b.hdr->err, kErrCoreCap);
            continue;
        }
        // start in the larger set: the first nearest-point search runs over the smaller one
        const bool swap = sj.m > si.m;
        const PointSet& sa = swap ? sj : si;
        const PointSet& sb = swap ? si : sj;
        int32_t p0[D];
        load_point<D>(sa, 0u, p0);
        uint32_t it = 0;
        const int yes = fast_merging_block<D, kWide, kCoopWaves>(sa, sb, p0, inst_T<kWide>(I), inst_Tm<kWide>(I),
                                                                  (double)I.eps, n_dist, it, sh);
        ++n_test;
        n_pts += si.m + sj.m;
        n_iter += it;
        max_it = it > max_it ? it : max_it;
        if (t0) {
            if (yes < 0) {
                atomicOr(&gv.b.hdr->err, kErrMergeRunaway);
            } else if (yes) {
                if (bfs && atomicCAS(&state[cj], kBfsNew, kBfsClassified) == kBfsNew)
                    next[atomicAdd(&cnt[2], 1u)] = cj;
                (void)uf_union_from(parent, uf_find(parent, ri), uf_find(parent, rj));
            }
        }
        n_yes += yes > 0 ? 1u : 0u;
    }
    // pair counts once per workgroup, distance evaluations once per wave
    if (stats && lane == 0) {
        if (t0)
            flush_stats(stats, blockIdx.x, 0ull, n_skip, n_test, n_yes, n_iter, max_it, n_dist, n_pts);
        else
            flush_stats(stats, blockIdx.x, 0ull, 0ull, 0ull, 0ull, 0ull, 0ull, n_dist, 0ull);
    }
}

hipError_t launch_huge_scan(const GridView& g, const CoreOut& c, const uint64_t* nei_off, unsigned long long* sum,
                            hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    huge_scan_kernel<<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(g.ncell_dev, c.core_cnt, nei_off, sum);
    return hipGetLastError();
}

hipError_t launch_merge_huge(const GridView& g, const CoreOut& c, const HugeQueue& huge, uint64_t* slabs,
                             uint32_t words, uint32_t blocks, bool bfs, bool wide, uint32_t* state, uint32_t* next,
                             uint32_t* cnt, uint32_t* parent, MergeStats* stats, hipStream_t st) {
    if (!huge.pairs || blocks == 0) return hipSuccess;
    const dim3 grid(blocks), threads(kCoopWaves * kWave);
    if (wide)
        GD_DISPATCH_D(g.D, (merge_heavy_kernel<D, true><<<grid, threads, 0, st>>>(
                               g, c, huge, slabs, words, bfs ? 1 : 0, state, next, cnt, parent, stats)));
    else
        GD_DISPATCH_D(g.D, (merge_heavy_kernel<D, false><<<grid, threads, 0, st>>>(
                               g, c, huge, slabs, words, bfs ? 1 : 0, state, next, cnt, parent, stats)));
    return hipGetLastError();
}

// Caller's d x m structure-of-arrays points to padded rows.
template <int D>
__global__ __launch_bounds__(kBlock) void soa_rows_kernel(const int32_t* __restrict__ pts, int64_t m,
                                                          int32_t* __restrict__ rows) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= m) return;
    int32_t y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) y[k] = pts[(int64_t)k * m + i];
    store_row<D>(rows, i, y);
}

// FastMerging on caller-given pairs of point runs (one wave per pair).
template <int D, bool kWide>
__global__ __launch_bounds__(kBlock) void merge_pairs_kernel(const int32_t* __restrict__ pts,
                                                             const uint32_t* __restrict__ pairs, int64_t npairs,
                                                             uint64_t T64, double eps, uint32_t words,
                                                             uint8_t* __restrict__ answers, uint32_t* iterations) {
    extern __shared__ uint64_t smem[];
    const int wpb = (int)(blockDim.x / kWave);
    const int w = wave_id();
    const int64_t r = block_id() * wpb + w;
    if (r >= npairs) return;
    PointSet a{pts, pairs[4 * r], pairs[4 * r + 1], smem + (int64_t)w * 2 * words, 0};
    PointSet b{pts, pairs[4 * r + 2], pairs[4 * r + 3], smem + (int64_t)w * 2 * words + words, 0};
    a.words = (a.m + kWave - 1) / kWave;
    b.words = (b.m + kWave - 1) / kWave;
    unsigned long long nd = 0;
    uint32_t it = 0;
    const typename Dist<kWide>::T T = (typename Dist<kWide>::T)T64;
    const int yes = fast_merging<D, kWide>(a, b, 0u, T, T, eps, nd, it);
    if (lane_id() == 0) {
        answers[r] = yes < 0 ? 2 : (uint8_t)yes;
        if (iterations) iterations[r] = it;
    }
}

hipError_t launch_merge_pairs(const int32_t* pts, int64_t m, int d, int32_t* rows, const uint32_t* pairs,
                              int64_t npairs, int64_t eps, uint32_t max_count, uint8_t* answers, uint32_t* iterations,
                              hipStream_t st) {
    if (npairs == 0) return hipSuccess;
    if (m > 0) GD_DISPATCH_D(d, (soa_rows_kernel<D><<<dim3(grid_for(m)), dim3(kBlock), 0, st>>>(pts, m, rows)));
    const uint32_t words = (max_count + kWave - 1) / kWave;
    int wpb = kWavesPerBlock;
    size_t lds = (size_t)wpb * 2 * words * sizeof(uint64_t);
    if (lds > 65536) {
        wpb = 1;
        lds = (size_t)2 * words * sizeof(uint64_t);
    }
    if (lds > 65536) return hipErrorInvalidValue;
    const dim3 blocks = grid_of((npairs + wpb - 1) / wpb);
    if (eps > GD_EPS_MAX)
        GD_DISPATCH_D(d, (merge_pairs_kernel<D, true><<<blocks, dim3(wpb * kWave), lds, st>>>(
                             rows, pairs, npairs, (uint64_t)(eps * eps), (double)eps, words, answers, iterations)));
    else
        GD_DISPATCH_D(d, (merge_pairs_kernel<D, false><<<blocks, dim3(wpb * kWave), lds, st>>>(
                             rows, pairs, npairs, (uint64_t)(eps * eps), (double)eps, words, answers, iterations)));
    return hipGetLastError();
}

// The smallest core index per union-find root.  Neighbouring grids mostly
// share a root, so the lanes holding the first lane's root reduce first and
// add one atomic; the rest add their own.
__global__ __launch_bounds__(kBlock) void root_min_kernel(const uint32_t* ncell, const uint32_t* core_cnt,
                                                          const uint32_t* cell_min_core, uint32_t* parent,
                                                          uint32_t* root_min) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool v = c < (int64_t)*ncell && core_cnt[c] != 0;
    const uint32_t r = v ? uf_find(parent, (uint32_t)c) : kNone;
    const uint32_t m = v ? cell_min_core[c] : kNone;
    const uint64_t valid = ballot(v);
    if (!valid) return;
    const uint32_t r0 = readlane(r, ffs64(valid));
    const bool same = v && r == r0;
    const uint32_t m0 = (uint32_t)wave_min_u64(same ? (uint64_t)m : ~0ull);
    if (lane_id() == ffs64(valid)) atomicMin(&root_min[r0], m0);
    if (v && !same) atomicMin(&root_min[r], m);
}

__global__ __launch_bounds__(kBlock) void cell_label_kernel(const uint32_t* ncell, const uint32_t* core_cnt,
                                                            uint32_t* parent, const uint32_t* root_min,
                                                            int32_t* cell_label) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= (int64_t)*ncell) return;
    cell_label[c] = core_cnt[c] == 0 ? -1 : (int32_t)root_min[uf_find(parent, (uint32_t)c)];
}

hipError_t launch_labels(const GridView& g, const CoreOut& c, uint32_t* parent, uint32_t* root_min,
                         int32_t* cell_label, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    // root_min was cleared to kNone with the core-grid list (launch_ldf_order)
    root_min_kernel<<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(g.ncell_dev, c.core_cnt, c.cell_min_core,
                                                                      parent, root_min);
    cell_label_kernel<<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(g.ncell_dev, c.core_cnt, parent, root_min,
                                                                        cell_label);
    return hipGetLastError();
}

}  // namespace gd
