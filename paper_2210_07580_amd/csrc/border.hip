// Border and noise points (Section 3.2 last step; Section 4.4 step 4) and
// the output in input order.
//
// One wave per grid.  Core points take their grid's cluster label.  A
// non-core point joins the cluster of its lowest-index core neighbour: the
// candidates are the grid's own core points (all within eps, the smallest
// index is precomputed) and the core points of Nei(g).  The wave streams the
// core sets of Nei(g) as one flat list (as in core marking),
// skipping grids whose smallest core index cannot improve any open query;
// for each non-core query a ballot finds the candidates within eps and a
// wave minimum over (input index << 32 | label) keeps the lowest index.
#include "launch.hpp"
#include "scan.hpp"

namespace gd {

template <int D>
__global__ __launch_bounds__(kBlock) void output_kernel(GridView gv, CoreOut co, const uint64_t* __restrict__ nei_off,
                                                        const uint32_t* __restrict__ nei,
                                                        const int32_t* __restrict__ cell_label) {
    __shared__ uint32_t s_start[kWavesPerBlock][kWave];
    __shared__ uint32_t s_excl[kWavesPerBlock][kWave];
    __shared__ int32_t s_lab[kWavesPerBlock][kWave];
    const int w = wave_id(), lane = lane_id();
    const int64_t c = (int64_t)blockIdx.x * kWavesPerBlock + w;
    if (c >= (int64_t)*gv.ncell_dev) return;
    const Inst& I = cell_inst(gv, c);
    const uint32_t off = (uint32_t)I.off;  // cluster ids and output slots are local to the instance
    int32_t* __restrict__ labels = I.labels;
    uint8_t* __restrict__ core_flags = I.core;
    const uint32_t st = gv.cell_start[c];
    const uint32_t k = gv.cell_start[c + 1] - st;
    const int32_t own_label = cell_label[c];
    const uint32_t own_min = co.cell_min_core[c];
    const uint32_t T = I.T;
    const uint64_t own_best = own_min == kNone ? ~0ull : (((uint64_t)own_min << 32) | (uint32_t)own_label);
    const uint64_t e0 = nei_off[c], e1 = nei_off[c + 1];
    for (uint32_t qb = 0; qb < k; qb += kWave) {
        const uint32_t s = st + qb + lane;
        const bool v = qb + lane < k;
        const uint8_t isc = v ? co.core[s] : 1;
        if (v && isc) {
            const uint32_t o = gv.sidx[s] - off;
            labels[o] = own_label - (int32_t)off;
            core_flags[o] = 1;
        }
        uint64_t open = ballot(v && !isc);  // non-core queries of this batch
        if (!open) continue;
        int32_t qx[D];
        load_row<D>(gv.crd, v ? s : st, qx);
        uint64_t best = own_best;  // lane i: best candidate of query i
        for (uint64_t e = e0; e < e1; e += kWave) {
            // largest best among open queries: grids whose smallest core index is not below it cannot help
            const uint64_t worst = ~wave_min_u64(((open >> lane) & 1ull) ? ~best : ~0ull);
            const uint32_t worst_idx = (uint32_t)(worst >> 32);
            const uint64_t idx = e + lane;
            uint32_t cs = 0, cn = 0;
            int32_t lab = -1;
            if (idx < e1) {
                const uint32_t cc = nei[idx];
                const uint32_t mc = co.cell_min_core[cc];
                if (mc != kNone && (worst == ~0ull || mc < worst_idx)) {
                    cs = co.core_begin[cc];
                    cn = co.core_cnt[cc];
                    lab = cell_label[cc];
                }
            }
            const uint32_t incl = wave_incl_scan(cn);
            const uint32_t tot = __shfl(incl, kWave - 1);
            if (tot == 0) continue;
            s_start[w][lane] = cs;
            s_excl[w][lane] = incl - cn;
            s_lab[w][lane] = lab;
            wave_sync();
            for (uint32_t t0 = 0; t0 < tot; t0 += kWave) {
                const uint32_t t = t0 + lane;
                const bool tv = t < tot;
                int j = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1)
                    if (s_excl[w][j + step] <= t) j += step;
                const uint32_t q = s_start[w][j] + (t - s_excl[w][j]);
                int32_t y[D];
                load_row<D>(co.ccrd, tv ? q : 0u, y);
                const uint64_t cand = tv ? (((uint64_t)co.corig[q] << 32) | (uint32_t)s_lab[w][j]) : ~0ull;
                uint64_t act = open;
                while (act) {
                    const int qi = ffs64(act);
                    act &= act - 1ull;
                    uint32_t dd = 0;
#pragma unroll
                    for (int jj = 0; jj < D; ++jj) dd += sq24(y[jj], readlane(qx[jj], qi));
                    const bool in = tv && dd <= T;
                    if (ballot(in)) {
                        const uint64_t m = wave_min_u64(in ? cand : ~0ull);
                        if (lane == qi && m < best) best = m;
                    }
                }
            }
            wave_sync();
        }
        if (v && !isc) {
            const uint32_t o = gv.sidx[s] - off;
            labels[o] = best == ~0ull ? -1 : (int32_t)((uint32_t)best - off);
            core_flags[o] = 0;
        }
    }
}

hipError_t launch_output(const GridView& g, const CoreOut& c, const uint64_t* nei_off, const uint32_t* nei,
                         const int32_t* cell_label, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    const unsigned blocks = grid_for(g.ncell, kWavesPerBlock);
    GD_DISPATCH_D(g.D, (output_kernel<D><<<dim3(blocks), dim3(kBlock), 0, st>>>(g, c, nei_off, nei, cell_label)));
    return hipGetLastError();
}

}  // namespace gd
