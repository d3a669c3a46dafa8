// Core points (Definition 1; identified "like G13", Section 3.2 and Section
// 4.4 step 2) and the per-grid core sets s_i used by the merge (Section
// 4.3.1), plus the low-density-first order of the LDF variant (Section 5.2).
//
// A core set is a run of point rows (see CoreOut): a grid whose points are
// all core uses its sorted rows as they are, so only grids that mix core and
// non-core points copy anything.
//
// Marking runs one wave per grid.  A grid with at least MinPts points is all
// core (its diameter is below eps).  In a sparser grid every point already
// has the grid's own points as neighbours; the wave then streams the points
// of Nei(g), nearest grids first, as one flat list: each lane owns one
// neighbour grid of a 64-grid chunk, a wave prefix sum of their sizes maps
// every flat item to its grid (binary search over 64 LDS entries), and each
// lane loads one candidate point per step.  The grid's own points are the
// queries: for each still-open query the wave evaluates 64 candidates at
// once, counts the hits with one ballot + popcount, and closes the query as
// soon as its count reaches MinPts (early exit).
#include "launch.hpp"
#include "radix.hpp"

namespace gd {

// Squared distance of two points of neighbouring grids: every coordinate
// difference is below 2.13 eps < 2^16 in magnitude, so each square is an
// exact unsigned 24-bit product, and the sum (below 9 eps^2 < 2^32 for
// eps <= 21845) is exact in unsigned 32-bit arithmetic.
// Above that bound (the wide path) the sum is taken in 64 bits.
template <int D, bool kWide>
__device__ __forceinline__ typename Dist<kWide>::T sqdist_nb(const int32_t (&a)[D], const int32_t (&b)[D]) {
    typename Dist<kWide>::T dd = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) dd += sqd<kWide>(a[j], b[j]);
    return dd;
}

// Packed form for small eps: points of neighbouring grids differ by less
// than (2 + sqrt(d - 1)) eps / sqrt(d) <= 2.13 eps per coordinate (the key
// offsets of Eq. (2) bound |k_j - k'_j| by 1 + sqrt(d - 1)), so for
// eps <= kPackedEpsMax every difference fits a signed 16-bit half and the
// squared distance (at most d (2.13 eps)^2 < 2^31) is exact in 32 bits.  Two
// coordinates share a word (low 16 bits of each; a 16-bit difference of the
// low halves is the exact difference when that is below 2^15), one packed
// subtraction and one two-term dot product handle both; an odd last
// coordinate stays a full word.

typedef short short2_t __attribute__((ext_vector_type(2)));

template <int D>
constexpr int packed_words() { return (D + 1) / 2; }

template <int D>
__device__ __forceinline__ void pack_row(const int32_t (&x)[D], int32_t (&p)[packed_words<D>()]) {
#pragma unroll
    for (int w = 0; w < D / 2; ++w) p[w] = (int32_t)(((uint32_t)x[2 * w] & 0xFFFFu) | ((uint32_t)x[2 * w + 1] << 16));
    if constexpr (D & 1) p[D / 2] = x[D - 1];
}

template <int D>
__device__ __forceinline__ uint32_t sqdist_pk(const int32_t (&a)[packed_words<D>()],
                                              const int32_t (&b)[packed_words<D>()]) {
    int32_t acc = 0;
#pragma unroll
    for (int w = 0; w < D / 2; ++w) {
        const short2_t t = __builtin_bit_cast(short2_t, a[w]) - __builtin_bit_cast(short2_t, b[w]);
        acc = __builtin_amdgcn_sdot2(t, t, acc, false);
    }
    if constexpr (D & 1) {
        const int32_t t = a[D / 2] - b[D / 2];
        acc = __mul24(t, t) + acc;
    }
    return (uint32_t)acc;
}

// R: candidate rows per lane per step.  The slowest grids stream dozens of
// steps one after another, each a chain of dependent rounds, so with a large
// MinPts (a query needs more hits than one 64-candidate step can give) a
// step takes two rows; with a small MinPts most queries close within the
// first 64 candidates and a second row would only add distance tests.
template <int D, bool kStats, bool kPacked, int R, bool kWide, bool kPrune>
__global__ __launch_bounds__(kBlock) void core_mark_kernel(GridView gv, const uint64_t* __restrict__ nei_off,
                                                           const uint32_t* __restrict__ nei, uint8_t* __restrict__ core,
                                                           uint32_t* __restrict__ core_cnt, CoreStats* stats) {
    constexpr int PW = packed_words<D>();
    constexpr int S = row_stride(D);
    __shared__ uint32_t s_start[kWavesPerBlock][kWave];
    __shared__ uint32_t s_excl[kWavesPerBlock][kWave];
    __shared__ __align__(16) int32_t s_q[kWavesPerBlock][kWave * S];  // the query rows of the batch
    const int w = wave_id(), lane = lane_id();
    const int64_t c = xcd_runs<16>(block_id(), block_count()) * kWavesPerBlock + w;
    if (c >= (int64_t)*gv.ncell_dev) return;
    // every load that depends on c alone is issued before the first use
    const Inst& I = cell_inst(gv, c);
    const uint32_t st = gv.cell_start[c];
    const uint32_t en = gv.cell_start[c + 1];
    const uint64_t e0 = nei_off[c], e1 = nei_off[c + 1];
    const uint32_t minpts = (uint32_t)I.minpts;
    const typename Dist<kWide>::T T = inst_T<kWide>(I);
    const uint32_t k = en - st;
    if (kPacked && I.eps > kPackedEpsMax) {
        // a replayed graph met a larger eps than it was captured for: the
        // packed differences could wrap, so the run is discarded
        if (lane == 0) atomicOr(&gv.b.hdr->err, kErrPlan);
        return;
    }
    if (k >= minpts) {
        for (uint32_t i = lane; i < k; i += kWave) core[st + i] = 1;
        if (lane == 0) core_cnt[c] = k;
        return;
    }
    const uint32_t need = minpts - k;
    const double side = kPrune && D <= 4 ? (double)I.eps / sqrt((double)I.d) : 0.0;
    const double lim = (double)I.eps * (double)I.eps * (1.0 + 1e-9) + 1.0;
    unsigned long long ndist = 0, npts = 0, ncells = 0;
    uint32_t m = 0;
    for (uint32_t qb = 0; qb < k; qb += kWave) {
        const uint32_t nq = min((uint32_t)kWave, k - qb);
        uint64_t active = nq == (uint32_t)kWave ? ~0ull : ((1ull << nq) - 1ull);
        int32_t qx[D];
        {
            load_row<D>(gv.crd, (uint32_t)lane < nq ? st + qb + lane : st, qx);
            if constexpr (kPacked) {
                int32_t pq[PW];
                pack_row<D>(qx, pq);
                store_row<PW>(s_q[w], lane, pq);
            } else {
                store_row<D>(s_q[w], lane, qx);
            }
        }
        uint32_t mycnt = 0;  // lane i: hits of query i
        for (uint64_t e = e0; e < e1 && active; e += kWave) {
            const uint64_t idx = e + lane;
            const bool v = idx < e1;
            const uint32_t cc = v ? nei[idx] : 0u;
            const uint32_t cs = v ? gv.cell_start[cc] : 0u;
            uint32_t cn = v ? gv.cell_start[cc + 1] - cs : 0u;
            if constexpr (kPrune && D <= 4) {
                // kPrune (low d, grids of a thousand points and more on
                // average): a grid of 16 steps or more is dropped when no
                // open query comes within eps of its cell, since the noise
                // points of a sparse grid stream every neighbour
                if (cn >= 16u * kWave && !cell_near<D>(gv, cc, active, qx, side, lim)) cn = 0;
            }
            const uint32_t incl = wave_incl_scan(cn);
            const uint32_t tot = __shfl(incl, kWave - 1);
            s_start[w][lane] = cs;
            s_excl[w][lane] = incl - cn;
            wave_sync();
            // row of flat candidate t (t < tot): binary search over the
            // chunk's 64 grids
            auto cand_row = [&](uint32_t t) -> uint32_t {
                int j = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1)
                    if (s_excl[w][j + step] <= t) j += step;
                return s_start[w][j] + (t - s_excl[w][j]);
            };
            // R candidates per lane per step (64 R per step), and the next
            // step's candidates load while this one is evaluated
            int32_t y[R][D];
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const uint32_t t = (uint32_t)(u * kWave + lane);
                load_row<D>(gv.crd, t < tot ? cand_row(t) : st, y[u]);
            }
            for (uint32_t t0 = 0; t0 < tot && active; t0 += R * kWave) {
                uint64_t tvm[R];
#pragma unroll
                for (int u = 0; u < R; ++u) tvm[u] = ballot(t0 + u * kWave + lane < tot);
                int32_t yn[R][D];
#pragma unroll
                for (int u = 0; u < R; ++u) {
                    const uint32_t tn = t0 + (R + u) * kWave + lane;
                    load_row<D>(gv.crd, tn < tot ? cand_row(tn) : st, yn[u]);
                }
                int32_t yp[R][PW];
                if constexpr (kPacked) {
#pragma unroll
                    for (int u = 0; u < R; ++u) pack_row<D>(y[u], yp[u]);
                }
                // every open query against the step's candidates, two queries
                // per round so their LDS reads overlap: the query row comes
                // from LDS (one broadcast read), lane qi keeps query qi's
                // hits; counts and closings are folded in once per step
                const uint64_t act0 = uniform64(active);
                uint32_t step_hits = 0;
                for (uint64_t act = act0; act;) {
                    const int qa = ffs64(act);
                    act &= act - 1ull;
                    const int qb2 = act ? ffs64(act) : qa;
                    act &= act - 1ull;
                    uint32_t ha = 0, hb = 0;
                    if constexpr (kPacked) {
                        int32_t pa[PW], pb[PW];
                        load_row<PW>(s_q[w], qa, pa);
                        load_row<PW>(s_q[w], qb2, pb);
#pragma unroll
                        for (int u = 0; u < R; ++u) {
                            ha += (uint32_t)popc64(ballot(sqdist_pk<D>(yp[u], pa) <= T) & tvm[u]);
                            hb += (uint32_t)popc64(ballot(sqdist_pk<D>(yp[u], pb) <= T) & tvm[u]);
                        }
                    } else {
                        int32_t pa[D], pb[D];
                        load_row<D>(s_q[w], qa, pa);
                        load_row<D>(s_q[w], qb2, pb);
#pragma unroll
                        for (int u = 0; u < R; ++u) {
                            ha += (uint32_t)popc64(ballot(sqdist_nb<D, kWide>(y[u], pa) <= T) & tvm[u]);
                            hb += (uint32_t)popc64(ballot(sqdist_nb<D, kWide>(y[u], pb) <= T) & tvm[u]);
                        }
                    }
                    step_hits = lane == qa ? ha : step_hits;
                    step_hits = lane == qb2 ? hb : step_hits;
                    if constexpr (kStats) ndist += (qb2 != qa ? 2u : 1u) * min(tot - t0, (uint32_t)(R * kWave));
                }
                mycnt += step_hits;
                active = act0 & ~ballot(((act0 >> lane) & 1ull) && mycnt >= need);
                if constexpr (kStats) npts += min(tot - t0, (uint32_t)(R * kWave));
#pragma unroll
                for (int u = 0; u < R; ++u)
#pragma unroll
                    for (int j = 0; j < D; ++j) y[u][j] = yn[u][j];
            }
            if constexpr (kStats) ncells += (unsigned long long)min(e1 - e, (uint64_t)kWave);
            wave_sync();
        }
        const bool is_core = (uint32_t)lane < nq && !((active >> lane) & 1ull);
        if ((uint32_t)lane < nq) core[st + qb + lane] = is_core ? 1 : 0;
        m += (uint32_t)popc64(ballot(is_core));
    }
    if (lane == 0) {
        core_cnt[c] = m;
        if constexpr (kStats) {
            CoreStats& sl = stats[c & (kStatSlots - 1)];
            atomicAdd(&sl.dists, ndist);
            atomicAdd(&sl.points, npts);
            atomicAdd(&sl.grids, ncells);
        }
    }
}

template <bool kStats, bool kPacked, int R, bool kWide>
hipError_t launch_core_mark_as(const GridView& g, const uint64_t* nei_off, const uint32_t* nei, uint8_t* core,
                               uint32_t* core_cnt, CoreStats* stats, bool prune, hipStream_t st) {
    const unsigned blocks = grid_for(g.ncell, kWavesPerBlock);
    if (prune)
        GD_DISPATCH_D(g.D, (core_mark_kernel<D, kStats, kPacked, R, kWide, true><<<grid_of(blocks), dim3(kBlock), 0,
                                                                                  st>>>(g, nei_off, nei, core,
                                                                                        core_cnt, stats)));
    else
        GD_DISPATCH_D(g.D, (core_mark_kernel<D, kStats, kPacked, R, kWide, false><<<grid_of(blocks), dim3(kBlock), 0,
                                                                                   st>>>(g, nei_off, nei, core,
                                                                                         core_cnt, stats)));
    return hipGetLastError();
}

hipError_t launch_core_mark(const GridView& g, const uint64_t* nei_off, const uint32_t* nei, uint8_t* core,
                            uint32_t* core_cnt, CoreStats* stats, int64_t max_eps, int64_t min_minpts, bool prune,
                            hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    const bool packed = core_mark_packed(max_eps);
    const bool two = min_minpts > kWave / 2;
    prune = prune && g.D <= 4;
    // the counting variant takes the same steps as the timed one
    if (max_eps > GD_EPS_MAX) {  // 64-bit distances, one row per step
        if (stats) return launch_core_mark_as<true, false, 1, true>(g, nei_off, nei, core, core_cnt, stats, prune, st);
        return launch_core_mark_as<false, false, 1, true>(g, nei_off, nei, core, core_cnt, stats, prune, st);
    }
    if (stats && two) return launch_core_mark_as<true, false, 2, false>(g, nei_off, nei, core, core_cnt, stats, prune, st);
    if (stats) return launch_core_mark_as<true, false, 1, false>(g, nei_off, nei, core, core_cnt, stats, prune, st);
    if (packed && two) return launch_core_mark_as<false, true, 2, false>(g, nei_off, nei, core, core_cnt, stats, prune, st);
    if (packed) return launch_core_mark_as<false, true, 1, false>(g, nei_off, nei, core, core_cnt, stats, prune, st);
    if (two) return launch_core_mark_as<false, false, 2, false>(g, nei_off, nei, core, core_cnt, stats, prune, st);
    return launch_core_mark_as<false, false, 1, false>(g, nei_off, nei, core, core_cnt, stats, prune, st);
}

// Side rows of grid c: its core count if it also holds non-core points.
struct SideRows {
    const uint32_t* cnt;
    const uint32_t* cell_start;
    const uint32_t* ncell;
    __device__ uint32_t operator()(int64_t c) const {
        if (c >= (int64_t)*ncell) return 0u;
        const uint32_t m = cnt[c];
        return (m != 0 && m != cell_start[c + 1] - cell_start[c]) ? m : 0u;
    }
};

// One thread per grid: where its core set starts, the smallest input index
// of its core points (grids without side rows), and the header counts.  The
// counts are reduced per workgroup and written to part[] (five words per
// workgroup), then summed by core_counts_fold: atomics from every wave to
// five addresses serialise on grids by the million.
__global__ __launch_bounds__(kBlock) void core_cells_kernel(GridView gv, CoreOut co, uint32_t* part) {
    __shared__ uint32_t red[5][kWavesPerBlock];
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool v = c < (int64_t)*gv.ncell_dev;
    uint32_t cnt = 0, size = 0, minpts = 0;
    if (v) {
        const uint32_t st = gv.cell_start[c];
        cnt = co.core_cnt[c];
        size = gv.cell_start[c + 1] - st;
        minpts = (uint32_t)cell_inst(gv, c).minpts;
        const bool side = cnt != 0 && cnt != size;
        co.core_begin[c] = side ? (uint32_t)gv.n + co.side_off[c] : st;
        if (!side) co.cell_min_core[c] = cnt ? gv.sidx[st] : kNone;
    }
    const uint32_t has = (uint32_t)popc64(ballot(v && cnt > 0));
    const uint32_t dense = (uint32_t)popc64(ballot(v && size >= minpts));
    const uint32_t tiny = (uint32_t)popc64(ballot(v && cnt > 0 && cnt <= kTinyCore));
    const uint32_t mx = wave_max_u32(cnt);
    const uint32_t tot = wave_sum(cnt);
    const int w = wave_id();
    if (lane_id() == 0) {
        red[0][w] = tot;
        red[1][w] = has;
        red[2][w] = mx;
        red[3][w] = dense;
        red[4][w] = tiny;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        uint32_t a = 0;
        for (int ww = 0; ww < kWavesPerBlock; ++ww)
            a = threadIdx.x == 2 ? max(a, red[2][ww]) : a + red[threadIdx.x][ww];
        part[(int64_t)blockIdx.x * 5 + threadIdx.x] = a;
    }
}

// counts[0..4] from the per-workgroup words of core_cells_kernel, by one
// workgroup (the first of the side copy, which needs no extra launch).
__device__ __forceinline__ void core_counts_fold(const uint32_t* part, int64_t blocks, uint32_t* counts) {
    __shared__ uint32_t red[5][kWavesPerBlock];
    uint32_t a[5] = {0, 0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < blocks; b += kBlock) {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const uint32_t x = part[b * 5 + k];
            a[k] = k == 2 ? max(a[k], x) : a[k] + x;
        }
    }
    const int w = wave_id();
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const uint32_t r = k == 2 ? wave_max_u32(a[k]) : wave_sum(a[k]);
        if (lane_id() == 0) red[k][w] = r;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        uint32_t r = 0;
        for (int ww = 0; ww < kWavesPerBlock; ++ww)
            r = threadIdx.x == 2 ? max(r, red[2][ww]) : r + red[threadIdx.x][ww];
        counts[threadIdx.x] = r;
    }
}

// One wave per grid holding both core and non-core points: copy its core
// rows, in sorted order, to the side area.  Workgroup 0 first folds the
// header counts (part, blocks: see core_cells_kernel).
template <int D>
__global__ __launch_bounds__(kBlock) void side_copy_kernel(GridView gv, CoreOut co, const uint32_t* part,
                                                           int64_t blocks) {
    if (blockIdx.x == 0) core_counts_fold(part, blocks, co.counts);
    // each wave checks 64 grids at once (one lane each) and copies only the
    // mixed ones: most grids need nothing, and a wave launched per grid would
    // spend the kernel on dispatching waves that exit at once
    const int lane = lane_id();
    const int64_t c0 = ((int64_t)blockIdx.x * kWavesPerBlock + wave_id()) * kWave;
    const int64_t ncell = *gv.ncell_dev;
    const int64_t cl = c0 + lane;
    uint32_t st_l = 0, k_l = 0, m_l = 0;
    if (cl < ncell) {
        st_l = gv.cell_start[cl];
        k_l = gv.cell_start[cl + 1] - st_l;
        m_l = co.core_cnt[cl];
    }
    uint64_t todo = ballot(cl < ncell && m_l != 0 && m_l != k_l);
    while (todo) {
        const int g = ffs64(todo);
        todo &= todo - 1ull;
        const int64_t c = c0 + g;
        const uint32_t st = readlane(st_l, g), k = readlane(k_l, g);
        const uint32_t base = (uint32_t)gv.n + co.side_off[c];
        uint32_t done = 0, first = kNone;
        for (uint32_t qb = 0; qb < k; qb += kWave) {
            const bool v = qb + lane < k;
            const bool f = v && co.core[st + qb + lane];
            const uint32_t orig = v ? gv.sidx[st + qb + lane] : 0u;
            const uint64_t bal = ballot(f);
            if (f) {
                const uint32_t r = base + done + (uint32_t)popc64(bal & lanemask_lt());
                int32_t y[D];
                load_row<D>(gv.crd, st + qb + lane, y);
                store_row<D>(co.ccrd, r, y);
                co.corig[r] = orig;
            }
            // sorted order within a grid is input order: the first core point has the smallest index
            if (first == kNone && bal) first = readlane(orig, ffs64(bal));
            done += (uint32_t)popc64(bal);
        }
        if (lane == 0) co.cell_min_core[c] = first;
    }
}

hipError_t launch_core_compact(const GridView& g, const CoreOut& c, uint32_t* partial, hipStream_t st) {
    if (g.ncell == 0) return fill<uint32_t>(c.counts, 5, 0u, st);
    hipError_t e;
    e = scan_exclusive<uint32_t>(SideRows{c.core_cnt, g.cell_start, g.ncell_dev}, g.ncell + 1, c.side_off,
                                 (uint32_t*)nullptr, partial, st);
    if (e != hipSuccess) return e;
    const unsigned nb = grid_for(g.ncell);
    core_cells_kernel<<<dim3(nb), dim3(kBlock), 0, st>>>(g, c, c.count_part);
    GD_DISPATCH_D(g.D, (side_copy_kernel<D><<<dim3(grid_for(g.ncell, kWavesPerBlock * kWave)), dim3(kBlock), 0, st>>>(
                           g, c, c.count_part, (int64_t)nb)));
    return hipGetLastError();
}

struct CoreCellFlag {
    const uint32_t* core_cnt;
    const uint32_t* ncell;
    __device__ uint32_t operator()(int64_t c) const { return c < (int64_t)*ncell && core_cnt[c] > 0; }
};

// Output of the core-grid scan: the list of core grids (and their counts as
// sort keys) in grid order, the merge record reset, every grid its own
// union-find root, and the per-root minima of the labelling step cleared.
struct CoreListWriter {
    const uint32_t* ncell;
    const uint32_t* core_cnt;
    uint32_t* list;
    uint32_t* keys;
    uint4* rec;
    uint32_t* parent;
    uint32_t* root_min;
    __device__ void operator()(int64_t c, uint32_t ex, uint32_t is_core) const {
        if (c >= (int64_t)*ncell) return;
        rec[c] = make_uint4(kNone, 0u, 0u, 0u);
        parent[c] = (uint32_t)c;
        root_min[c] = kNone;
        if (is_core) {
            list[ex] = (uint32_t)c;
            keys[ex] = core_cnt[c];
        }
    }
};

// The merge step's record of each core grid: rank in the visiting order,
// first row and size of its core set (one load instead of three).
__global__ __launch_bounds__(kBlock) void rank_kernel(const uint32_t* sorted, const uint32_t* m, CoreOut co,
                                                      uint4* rec) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r >= (int64_t)*m) return;
    const uint32_t c = sorted[r];
    rec[c] = make_uint4((uint32_t)r, co.core_begin[c], co.core_cnt[c], 0u);
}

hipError_t launch_ldf_order(const GridView& g, const CoreOut& c, bool by_count, int64_t ncc, int count_bits,
                            bool pad_tail, uint32_t* list, uint4* rank, uint32_t* parent, uint32_t* root_min,
                            uint32_t* keys_a, uint32_t* keys_b, uint32_t* vals_b, uint32_t* radix_scratch,
                            uint32_t* partial, uint32_t** sorted_list, hipStream_t st) {
    *sorted_list = list;
    if (g.ncell == 0) return hipSuccess;
    if (by_count && pad_tail && ncc > 0) {
        hipError_t e = fill<uint32_t>(keys_a, ncc, (uint32_t)((1ull << count_bits) - 1ull), st);
        if (e != hipSuccess) return e;
    }
    hipError_t e = scan_apply<uint32_t>(CoreCellFlag{c.core_cnt, g.ncell_dev}, g.ncell,
                                        CoreListWriter{g.ncell_dev, c.core_cnt, list, keys_a, rank, parent, root_min},
                                        (uint32_t*)nullptr, partial, st);
    if (e != hipSuccess) return e;
    if (by_count && ncc > 1) {
        RadixResult<uint32_t> res;
        e = radix_sort_pairs<uint32_t>(keys_a, list, keys_b, vals_b, ncc, count_bits, false, radix_scratch, st, &res);
        if (e != hipSuccess) return e;
        *sorted_list = res.vals;
    }
    if (ncc > 0) rank_kernel<<<dim3(grid_for(ncc)), dim3(kBlock), 0, st>>>(*sorted_list, &c.counts[1], c, rank);
    return hipGetLastError();
}

}  // namespace gd
