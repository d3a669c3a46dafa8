// Core points (Definition 1; identified "like G13", Section 3.2 and Section
// 4.4 step 2) and the per-grid core sets s_i used by the merge (Section
// 4.3.1), plus the low-density-first order of the LDF variant (Section 5.2).
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

template <int D>
__global__ __launch_bounds__(kBlock) void core_mark_kernel(GridView gv, const uint64_t* __restrict__ nei_off,
                                                           const uint32_t* __restrict__ nei, uint8_t* __restrict__ core,
                                                           unsigned long long* dist_counter) {
    __shared__ uint32_t s_start[kWavesPerBlock][kWave];
    __shared__ uint32_t s_excl[kWavesPerBlock][kWave];
    const int w = wave_id(), lane = lane_id();
    const int64_t c = (int64_t)blockIdx.x * kWavesPerBlock + w;
    if (c >= (int64_t)*gv.ncell_dev) return;
    const Inst& I = cell_inst(gv, c);
    const uint32_t st = gv.cell_start[c];
    const uint32_t k = gv.cell_start[c + 1] - st;
    const uint32_t minpts = (uint32_t)I.minpts;
    const int64_t n = gv.n;
    if (k >= minpts) {
        for (uint32_t i = lane; i < k; i += kWave) core[st + i] = 1;
        return;
    }
    const uint32_t need = minpts - k;
    const uint32_t T = I.T;
    const uint64_t e0 = nei_off[c], e1 = nei_off[c + 1];
    unsigned long long ndist = 0;
    for (uint32_t qb = 0; qb < k; qb += kWave) {
        const uint32_t nq = min((uint32_t)kWave, k - qb);
        uint64_t active = nq == (uint32_t)kWave ? ~0ull : ((1ull << nq) - 1ull);
        int32_t qx[D];
#pragma unroll
        for (int j = 0; j < D; ++j) qx[j] = (uint32_t)lane < nq ? gv.crd[(int64_t)j * n + st + qb + lane] : 0;
        uint32_t mycnt = 0;
        for (uint64_t e = e0; e < e1 && active; e += kWave) {
            const uint64_t idx = e + lane;
            const bool v = idx < e1;
            const uint32_t cc = v ? nei[idx] : 0u;
            const uint32_t cs = v ? gv.cell_start[cc] : 0u;
            const uint32_t cn = v ? gv.cell_start[cc + 1] - cs : 0u;
            const uint32_t incl = wave_incl_scan(cn);
            const uint32_t tot = __shfl(incl, kWave - 1);
            s_start[w][lane] = cs;
            s_excl[w][lane] = incl - cn;
            wave_sync();
            for (uint32_t t0 = 0; t0 < tot && active; t0 += kWave) {
                const uint32_t t = t0 + lane;
                const bool tv = t < tot;
                int j = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1)
                    if (s_excl[w][j + step] <= t) j += step;
                const uint32_t q = s_start[w][j] + (t - s_excl[w][j]);
                int32_t y[D];
#pragma unroll
                for (int jj = 0; jj < D; ++jj) y[jj] = tv ? gv.crd[(int64_t)jj * n + q] : 0;
                uint64_t act = active;
                const int nv = popc64(ballot(tv));
                while (act) {
                    const int qi = ffs64(act);
                    act &= act - 1ull;
                    uint32_t dd = 0;
#pragma unroll
                    for (int jj = 0; jj < D; ++jj) dd += sq24(y[jj], readlane(qx[jj], qi));
                    const uint32_t hits = (uint32_t)popc64(ballot(tv && dd <= T));
                    if (lane == qi) mycnt += hits;
                    if (readlane(mycnt, qi) >= need) active &= ~(1ull << qi);
                    ndist += (unsigned long long)nv;
                }
            }
            wave_sync();
        }
        if ((uint32_t)lane < nq) core[st + qb + lane] = ((active >> lane) & 1ull) ? 0 : 1;
    }
    if (dist_counter && lane == 0) atomicAdd(&dist_counter[c & (kStatSlots - 1)], ndist);
}

hipError_t launch_core_mark(const GridView& g, const uint64_t* nei_off, const uint32_t* nei, uint8_t* core,
                            unsigned long long* dist_counter, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    const unsigned blocks = grid_for(g.ncell, kWavesPerBlock);
    GD_DISPATCH_D(g.D, (core_mark_kernel<D><<<dim3(blocks), dim3(kBlock), 0, st>>>(g, nei_off, nei, core, dist_counter)));
    return hipGetLastError();
}

struct CoreFlag {
    const uint8_t* core;
    int64_t n;
    __device__ uint32_t operator()(int64_t i) const { return i < n ? (uint32_t)core[i] : 0u; }
};

__global__ __launch_bounds__(kBlock) void core_scatter_kernel(GridView gv, CoreOut co) {
    const int64_t s = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (s >= gv.n || !co.core[s]) return;
    const uint32_t pos = co.core_excl[s];
    for (int j = 0; j < gv.D; ++j) co.ccrd[(int64_t)pos * co.cstride + j] = gv.crd[(int64_t)j * gv.n + s];
    co.corig[pos] = gv.sidx[s];
}

__global__ __launch_bounds__(kBlock) void core_start_kernel(GridView gv, CoreOut co) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c > (int64_t)*gv.ncell_dev) return;
    co.core_start[c] = co.core_excl[gv.cell_start[c]];
}

__global__ __launch_bounds__(kBlock) void core_cells_kernel(GridView gv, CoreOut co) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool v = c < (int64_t)*gv.ncell_dev;
    uint32_t cnt = 0, size = 0, minpts = 0;
    if (v) {
        const uint32_t a = co.core_start[c];
        cnt = co.core_start[c + 1] - a;
        size = gv.cell_start[c + 1] - gv.cell_start[c];
        minpts = (uint32_t)cell_inst(gv, c).minpts;
        co.cell_min_core[c] = cnt ? co.corig[a] : kNone;
    }
    const uint64_t has = ballot(v && cnt > 0);
    const uint64_t dense = ballot(v && size >= minpts);
    const uint64_t tiny = ballot(v && cnt > 0 && cnt <= kTinyCore);
    const uint32_t mx = wave_max_u32(cnt);
    if (lane_id() == 0) {
        if (has) atomicAdd(&co.counts[1], (uint32_t)popc64(has));
        if (dense) atomicAdd(&co.counts[3], (uint32_t)popc64(dense));
        if (tiny) atomicAdd(&co.counts[4], (uint32_t)popc64(tiny));
        if (mx) atomicMax(&co.counts[2], mx);
    }
}

hipError_t launch_core_compact(const GridView& g, const CoreOut& c, uint32_t* partial, hipStream_t st) {
    hipError_t e = fill<uint32_t>(c.counts, 5, 0u, st);
    if (e != hipSuccess) return e;
    // core_excl[n] = number of core points, also copied to counts[0]
    e = scan_exclusive<uint32_t>(CoreFlag{c.core, g.n}, g.n + 1, c.core_excl, c.counts, partial, st);
    if (e != hipSuccess) return e;
    if (g.n == 0) return hipSuccess;
    core_scatter_kernel<<<dim3(grid_for(g.n)), dim3(kBlock), 0, st>>>(g, c);
    core_start_kernel<<<dim3(grid_for(g.ncell + 1)), dim3(kBlock), 0, st>>>(g, c);
    core_cells_kernel<<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(g, c);
    return hipGetLastError();
}

struct CoreCellFlag {
    const uint32_t* core_start;
    const uint32_t* ncell;
    __device__ uint32_t operator()(int64_t c) const {
        return c < (int64_t)*ncell && core_start[c + 1] > core_start[c];
    }
};

__global__ __launch_bounds__(kBlock) void core_list_kernel(const uint32_t* ncell_dev, const uint32_t* core_start,
                                                           const uint32_t* excl, uint32_t* list, uint32_t* keys,
                                                           uint32_t* rank) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= (int64_t)*ncell_dev) return;
    const uint32_t cnt = core_start[c + 1] - core_start[c];
    rank[c] = kNone;
    if (cnt) {
        list[excl[c]] = (uint32_t)c;
        keys[excl[c]] = cnt;
    }
}

__global__ __launch_bounds__(kBlock) void rank_kernel(const uint32_t* sorted, int64_t m, uint32_t* rank) {
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (r < m) rank[sorted[r]] = (uint32_t)r;
}

hipError_t launch_ldf_order(const GridView& g, const CoreOut& c, bool by_count, int64_t ncc, int count_bits,
                            uint32_t* list, uint32_t* rank, uint32_t* keys_a, uint32_t* keys_b, uint32_t* vals_b,
                            uint32_t* radix_scratch, uint32_t* excl, uint32_t* partial, uint32_t** sorted_list,
                            hipStream_t st) {
    *sorted_list = list;
    if (g.ncell == 0) return hipSuccess;
    hipError_t e = scan_exclusive<uint32_t>(CoreCellFlag{c.core_start, g.ncell_dev}, g.ncell, excl,
                                            (uint32_t*)nullptr, partial, st);
    if (e != hipSuccess) return e;
    core_list_kernel<<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(g.ncell_dev, c.core_start, excl, list, keys_a,
                                                                      rank);
    if (by_count && ncc > 1) {
        RadixResult<uint32_t> res;
        e = radix_sort_pairs<uint32_t>(keys_a, list, keys_b, vals_b, ncc, count_bits, false, radix_scratch, st, &res);
        if (e != hipSuccess) return e;
        *sorted_list = res.vals;
    }
    if (ncc > 0) rank_kernel<<<dim3(grid_for(ncc)), dim3(kBlock), 0, st>>>(*sorted_list, ncc, rank);
    return hipGetLastError();
}

}  // namespace gd
