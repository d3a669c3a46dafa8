// Consumers that query their neighbouring grids themselves (walk.hpp)
// instead of reading materialised Nei(g) lists: core marking (Section 3.2,
// Section 4.4 step 2), the merging of tiny core sets (Section 4.3, Theorem 2)
// and border assignment (Section 4.4 step 4).
//
// With sparse grids in many dimensions the lists dwarf the data: at d = 5,
// eps / sqrt(d) grids hold one or two points each and every grid has
// hundreds of non-empty neighbours, so writing the lists and streaming them
// back costs far more than the tree walks that produce them.  Each consumer
// here walks the tree for its own grid, one thread per grid, and uses each
// neighbour the moment it is found:
//   core marking   - the grid's queries count hits over its neighbours' points
//                    and the walk stops once every query reached MinPts;
//   tiny merging   - a tiny core grid walks only the neighbours with a larger
//                    identifier (each unordered pair once, from its lower
//                    grid) and decides each pair of tiny core sets by their
//                    distances directly (FastMerging's answer, Theorem 2);
//   border points  - the grid's non-core points look for their lowest-index
//                    core neighbour over the whole neighbourhood.
// Pairs with a core set of more than kTinyCore points are merged by the list
// kernels, from lists built for those grids only.
#include "fastmerge.hpp"
#include "launch.hpp"
#include "walk.hpp"

namespace gd {

constexpr int kWalkQueries = 4;  // queries of one grid evaluated per walk

template <int D, bool kWide>
__device__ __forceinline__ typename Dist<kWide>::T sqdist_rows(const int32_t (&a)[D], const int32_t (&b)[D]) {
    typename Dist<kWide>::T dd = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) dd += sqd<kWide>(a[j], b[j]);
    return dd;
}

// Grid index of thread `tid`: blocks are spread over the XCDs in runs so that
// neighbouring grids, which read largely the same tree nodes and rows, share
// an L2 (only the speed depends on it).
__device__ __forceinline__ int64_t walk_grid(int64_t nblocks) {
    return xcd_runs<16>(blockIdx.x, nblocks) * kBlock + threadIdx.x;
}

template <int D, bool kStats, bool kWide>
__global__ __launch_bounds__(kBlock) void core_walk_kernel(GridView gv, TreeView t, uint8_t* __restrict__ core,
                                                           uint32_t* __restrict__ core_cnt, CoreStats* stats) {
    const int64_t c = walk_grid(gridDim.x);
    if (c >= (int64_t)*gv.ncell_dev) return;
    const Inst& I = cell_inst(gv, c);
    const uint32_t st = gv.cell_start[c];
    const uint32_t k = gv.cell_start[c + 1] - st;
    const uint32_t minpts = (uint32_t)I.minpts;
    if (k >= minpts) {  // a grid's diameter is below eps: all core
        for (uint32_t i = 0; i < k; ++i) core[st + i] = 1;
        core_cnt[c] = k;
        return;
    }
    const typename Dist<kWide>::T T = inst_T<kWide>(I);
    const uint32_t need = minpts - k;  // hits still needed beyond the own grid
    const int dk = I.d;
    int32_t g[D + 1];
    load_grid_key<D>(gv, c, g);
    unsigned long long ndist = 0, npts = 0, ngrids = 0;
    uint32_t m = 0;
    for (uint32_t qb = 0; qb < k; qb += kWalkQueries) {
        const uint32_t nq = min((uint32_t)kWalkQueries, k - qb);
        int32_t q[kWalkQueries][D];
        uint32_t hits[kWalkQueries];
        uint32_t open = (1u << nq) - 1u;
#pragma unroll
        for (int u = 0; u < kWalkQueries; ++u) {
            load_row<D>(gv.crd, st + qb + min((uint32_t)u, nq - 1), q[u]);
            hits[u] = 0;
        }
        auto visit = [&](uint32_t a, int) -> bool {
            if (a == (uint32_t)c) return true;
            const uint32_t cs = gv.cell_start[a], ce = gv.cell_start[a + 1];
            if constexpr (kStats) {
                ++ngrids;
                npts += ce - cs;
            }
            for (uint32_t r = cs; r < ce; ++r) {
                int32_t y[D];
                load_row<D>(gv.crd, r, y);
#pragma unroll
                for (int u = 0; u < kWalkQueries; ++u) {
                    if (!((open >> u) & 1u)) continue;
                    if constexpr (kStats) ++ndist;
                    if (sqdist_rows<D, kWide>(q[u], y) <= T && ++hits[u] >= need) open &= ~(1u << u);
                }
                if (!open) return false;  // every query reached MinPts
            }
            return true;
        };
        tree_walk<D>(t, g, dk, false, visit);
#pragma unroll
        for (int u = 0; u < kWalkQueries; ++u) {
            if ((uint32_t)u >= nq) continue;
            const bool is_core = hits[u] >= need;
            core[st + qb + u] = is_core ? 1 : 0;
            m += is_core ? 1u : 0u;
        }
    }
    core_cnt[c] = m;
    if constexpr (kStats) {
        CoreStats& sl = stats[c & (kStatSlots - 1)];
        atomicAdd(&sl.dists, ndist);
        atomicAdd(&sl.points, npts);
        atomicAdd(&sl.grids, ngrids);
    }
}

hipError_t launch_core_walk(const GridView& g, const TreeView& t, uint8_t* core, uint32_t* core_cnt, CoreStats* stats,
                            bool wide, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    const dim3 blocks(grid_for(g.ncell)), threads(kBlock);
    if (stats && wide)
        GD_DISPATCH_D(g.D, (core_walk_kernel<D, true, true><<<blocks, threads, 0, st>>>(g, t, core, core_cnt, stats)));
    else if (stats)
        GD_DISPATCH_D(g.D, (core_walk_kernel<D, true, false><<<blocks, threads, 0, st>>>(g, t, core, core_cnt, stats)));
    else if (wide)
        GD_DISPATCH_D(g.D, (core_walk_kernel<D, false, true><<<blocks, threads, 0, st>>>(g, t, core, core_cnt, stats)));
    else
        GD_DISPATCH_D(g.D, (core_walk_kernel<D, false, false><<<blocks, threads, 0, st>>>(g, t, core, core_cnt, stats)));
    return hipGetLastError();
}

// One thread per tiny core grid (at most kTinyCore core points), in the
// visiting order: every neighbour with a larger identifier that is also a
// tiny core grid is a candidate; a pair already in one set is skipped,
// otherwise its |s_i| x |s_j| distances decide it.
template <int D, bool kStats, bool kWide>
__global__ __launch_bounds__(kBlock) void merge_walk_kernel(GridView gv, CoreOut co, TreeView t,
                                                            const uint32_t* __restrict__ ldf, int64_t r1,
                                                            const uint32_t* split, uint32_t* parent,
                                                            MergeStats* stats) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= r1 || r >= (int64_t)co.counts[1] || (split && r >= (int64_t)*split)) return;
    const uint32_t ci = ldf[r];
    const uint32_t mi = co.core_cnt[ci];
    if (mi == 0 || mi > kTinyCore) return;
    const uint32_t bi = co.core_begin[ci];
    const Inst& I = cell_inst(gv, ci);
    const typename Dist<kWide>::T T = inst_Tm<kWide>(I);  // the merge's "yes" bound (eps^2 unless approximate)
    const int dk = I.d;
    int32_t pi[kTinyCore][D];
#pragma unroll
    for (int a = 0; a < (int)kTinyCore; ++a) load_row<D>(co.ccrd, bi + min((uint32_t)a, mi - 1), pi[a]);
    int32_t g[D + 1];
    load_grid_key<D>(gv, ci, g);
    unsigned long long n_pairs = 0, n_skip = 0, n_yes = 0, n_dist = 0, n_pts = 0;
    uint32_t ri = uf_find(parent, ci);  // root hint of g_i's set
    auto visit = [&](uint32_t cj, int) -> bool {
        const uint32_t mj = co.core_cnt[cj];
        if (mj == 0 || mj > kTinyCore) return true;
        const uint32_t rj = uf_find(parent, cj);
        if constexpr (kStats) ++n_pairs;
        if (rj == ri) {
            if constexpr (kStats) ++n_skip;
            return true;
        }
        const uint32_t bj = co.core_begin[cj];
        bool yes = false;
        for (uint32_t b = 0; b < mj && !yes; ++b) {
            int32_t y[D];
            load_row<D>(co.ccrd, bj + b, y);
#pragma unroll
            for (int a = 0; a < (int)kTinyCore; ++a)
                if ((uint32_t)a < mi) yes |= sqdist_rows<D, kWide>(pi[a], y) <= T;
        }
        if constexpr (kStats) {
            n_dist += (unsigned long long)mi * mj;
            n_pts += mi + mj;
        }
        if (yes) {
            if constexpr (kStats) ++n_yes;
            uf_union_from(parent, ri, rj);
            ri = uf_find(parent, ri);
        }
        return true;
    };
    tree_walk<D>(t, g, dk, true, visit);
    if constexpr (kStats) {
        // each direct test counts as one FastMerging iteration
        MergeStats* sl = stats + ((uint64_t)r & (kStatSlots - 1));
        const unsigned long long nt = n_pairs - n_skip;
        atomicAdd(&sl->pairs, n_pairs);
        atomicAdd(&sl->skipped, n_skip);
        atomicAdd(&sl->tests, nt);
        atomicAdd(&sl->yes, n_yes);
        atomicAdd(&sl->iters, nt);
        atomicMax(&sl->max_iters, nt ? 1ull : 0ull);
        atomicAdd(&sl->dists, n_dist);
        atomicAdd(&sl->set_points, n_pts);
    }
}

hipError_t launch_merge_walk(const GridView& g, const CoreOut& c, const TreeView& t, const uint32_t* ldf_list,
                             int64_t n_small, uint32_t* parent, MergeStats* stats, bool wide, hipStream_t st) {
    // n_small >= 0: the first n_small ranks are the tiny core grids; -2: as
    // many as the device count says
    const uint32_t* split = n_small == -2 ? &c.counts[4] : nullptr;
    const int64_t r1 = n_small >= 0 ? n_small : g.ncell;
    if (r1 <= 0) return hipSuccess;
    const dim3 blocks(grid_for(r1)), threads(kBlock);
    if (stats && wide)
        GD_DISPATCH_D(g.D, (merge_walk_kernel<D, true, true><<<blocks, threads, 0, st>>>(g, c, t, ldf_list, r1, split,
                                                                                        parent, stats)));
    else if (stats)
        GD_DISPATCH_D(g.D, (merge_walk_kernel<D, true, false><<<blocks, threads, 0, st>>>(g, c, t, ldf_list, r1, split,
                                                                                         parent, stats)));
    else if (wide)
        GD_DISPATCH_D(g.D, (merge_walk_kernel<D, false, true><<<blocks, threads, 0, st>>>(g, c, t, ldf_list, r1, split,
                                                                                         parent, stats)));
    else
        GD_DISPATCH_D(g.D, (merge_walk_kernel<D, false, false><<<blocks, threads, 0, st>>>(g, c, t, ldf_list, r1,
                                                                                          split, parent, stats)));
    return hipGetLastError();
}

// One thread per grid holding a non-core point: its core points take the
// grid's label, its non-core points the label of their lowest-index core
// neighbour (own grid first: all of its points are within eps), else -1.
template <int D, bool kWide>
__global__ __launch_bounds__(kBlock) void border_walk_kernel(GridView gv, CoreOut co, TreeView t,
                                                             const int32_t* __restrict__ cell_label) {
    const int64_t c = walk_grid(gridDim.x);
    if (c >= (int64_t)*gv.ncell_dev) return;
    const uint32_t st = gv.cell_start[c];
    const uint32_t k = gv.cell_start[c + 1] - st;
    if (co.core_cnt[c] == k) return;  // all core: written in input order by the hash pass
    const Inst& I = cell_inst(gv, c);
    const uint32_t off = (uint32_t)I.off;
    int32_t GD_GLOBAL* __restrict__ labels = as_global(I.labels);
    uint8_t GD_GLOBAL* __restrict__ core_flags = as_global(I.core);
    const int32_t own_label = cell_label[c];
    const uint32_t own_min = co.cell_min_core[c];
    const typename Dist<kWide>::T T = inst_T<kWide>(I);
    const int dk = I.d;
    const uint64_t own_best = own_min == kNone ? ~0ull : (((uint64_t)own_min << 32) | (uint32_t)own_label);
    int32_t g[D + 1];
    load_grid_key<D>(gv, c, g);
    // the grid's core points take its label as the scan passes them
    auto skip_core = [&](uint32_t& scan) {
        while (scan < k && co.core[st + scan]) {
            const uint32_t o = gv.sidx[st + scan] - off;
            labels[o] = own_label - (int32_t)off;
            core_flags[o] = 1;
            ++scan;
        }
    };
    uint32_t scan = 0;
    for (;;) {
        // the next (up to) kWalkQueries non-core points of the grid; every
        // slot index is a compile-time constant (filling the array through
        // a per-lane counter in this divergent loop, the first form, gave
        // positions past the grid's end when built for gfx950)
        uint32_t pos[kWalkQueries];
        int nq = 0;
#pragma unroll
        for (int u = 0; u < kWalkQueries; ++u) {
            skip_core(scan);
            pos[u] = st;
            if (scan < k) {
                pos[u] = st + scan;
                ++scan;
                nq = u + 1;
            }
        }
        if (nq == 0) break;
        int32_t q[kWalkQueries][D];
        uint64_t best[kWalkQueries];
#pragma unroll
        for (int u = 0; u < kWalkQueries; ++u) {
            load_row<D>(gv.crd, pos[u], q[u]);
            best[u] = own_best;
        }
        auto visit = [&](uint32_t a, int) -> bool {
            if (a == (uint32_t)c) return true;
            const uint32_t mc = co.cell_min_core[a];
            if (mc == kNone) return true;
            // a grid whose smallest core index is not below every open
            // query's best cannot improve any of them
            uint64_t worst = 0;
#pragma unroll
            for (int u = 0; u < kWalkQueries; ++u)
                if (u < nq) worst = best[u] > worst ? best[u] : worst;
            if (worst != ~0ull && mc >= (uint32_t)(worst >> 32)) return true;
            const uint32_t cs = co.core_begin[a], cn = co.core_cnt[a];
            const int32_t lab = cell_label[a];
            for (uint32_t r = cs; r < cs + cn; ++r) {
                int32_t y[D];
                load_row<D>(co.ccrd, r, y);
                const uint64_t cand = ((uint64_t)co.corig[r] << 32) | (uint32_t)lab;
#pragma unroll
                for (int u = 0; u < kWalkQueries; ++u)
                    if (u < nq && cand < best[u] && sqdist_rows<D, kWide>(q[u], y) <= T) best[u] = cand;
            }
            return true;
        };
        tree_walk<D>(t, g, dk, false, visit);
#pragma unroll
        for (int u = 0; u < kWalkQueries; ++u) {
            if (u >= nq) continue;
            const uint32_t o = gv.sidx[pos[u]] - off;
            labels[o] = best[u] == ~0ull ? -1 : (int32_t)((uint32_t)best[u] - off);
            core_flags[o] = 0;
        }
    }
}

hipError_t launch_border_walk(const GridView& g, const CoreOut& c, const TreeView& t, const int32_t* cell_label,
                              bool wide, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    const dim3 blocks(grid_for(g.ncell)), threads(kBlock);
    if (wide)
        GD_DISPATCH_D(g.D, (border_walk_kernel<D, true><<<blocks, threads, 0, st>>>(g, c, t, cell_label)));
    else
        GD_DISPATCH_D(g.D, (border_walk_kernel<D, false><<<blocks, threads, 0, st>>>(g, c, t, cell_label)));
    return hipGetLastError();
}

}  // namespace gd
