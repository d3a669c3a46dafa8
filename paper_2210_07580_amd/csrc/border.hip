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
//
// Writing in input order: grids whose points are all core (nearly every
// point in dense data) do not scatter their output through the sort
// permutation.  A hash table maps each grid's identifier to its label; one
// pass over the points in input order re-reads each point's identifier
// (kept from before the sort), looks the label up and writes labels and
// flags with coalesced stores.  Only grids holding a non-core point go
// through the wave-per-grid kernel, which writes through the permutation.
#include <algorithm>

#include "hash.hpp"
#include "launch.hpp"
#include "scan.hpp"

namespace gd {

constexpr int32_t kDeferred = -2;  // grid output written by the wave-per-grid kernel


template <typename K>
__global__ __launch_bounds__(kBlock) void hash_build_kernel(GridView gv, CoreOut co, const K* __restrict__ skeys,
                                                            const int32_t* __restrict__ cell_label,
                                                            HashSlot<K>* tab, int bits) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= (int64_t)*gv.ncell_dev) return;
    const uint32_t st = gv.cell_start[c];
    const uint32_t k = gv.cell_start[c + 1] - st;
    // only all-core grids go in: a missing identifier reads as deferred
    if (co.core_cnt[c] != k) return;
    grid_table_insert<K>(tab, bits, skeys[st], cell_label[c]);
}

// Points in input order, instance tiles as in the identifier pass, each
// tile split into `parts` workgroups of at most kOutputPart points (the
// lookups are latency-bound: with 4096-point tiles a call of 10M points
// left about one wave per slot and a long tail; 1024-point parts cut the
// pass by a tenth on such calls); each thread resolves U points at a time
// so that their loads overlap.  The identifier of input word w is
// w >> key_lo (key_lo > 0: packed rows in two-word keys).
constexpr int kOutputPart = 1024;
template <typename K>
__global__ __launch_bounds__(kBlock) void output_direct_kernel(Batch b, const K* __restrict__ keys,
                                                               const HashSlot<K>* __restrict__ tab, int bits,
                                                               int key_lo, int parts) {
    constexpr int U = 8;
    if (b.hdr->err & kErrPlan) return;  // a sync-free run that stopped early (its result is discarded)
    const uint32_t tile = blockIdx.x / (uint32_t)parts, part = blockIdx.x % (uint32_t)parts;
    const int k = tile_instance(b, tile);
    const Inst& I = b.inst[k];
    const int64_t sub = ((int64_t)b.tile_pts + parts - 1) / parts;
    const int64_t t0 = (int64_t)(tile - I.tile0) * b.tile_pts;
    const int64_t lo = t0 + (int64_t)part * sub;
    const int64_t hi = min(I.n, min(lo + sub, t0 + (int64_t)b.tile_pts));
    const int bbits = bits - kBucketShift<K>;
    const uint64_t bmask = (1ull << bbits) - 1ull;
    const int32_t off = (int32_t)I.off;
    int32_t GD_GLOBAL* __restrict__ labels = as_global(I.labels);
    uint8_t GD_GLOBAL* __restrict__ flags = as_global(I.core);
    const int32_t special = tab[1ull << bits].val;
    for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += U * kBlock) {
        K key[U];
        uint64_t bk[U];
        uint4 q[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + (int64_t)u * kBlock;
            key[u] = i < hi ? keys[I.off + i] >> key_lo : ~K(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            bk[u] = hash_bucket(key[u], bbits);
            if (key[u] != ~K(0)) q[u] = load_bucket(tab, bk[u]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = i0 + (int64_t)u * kBlock;
            if (i >= hi) continue;
            int32_t val = kDeferred;
            if (key[u] == ~K(0)) {
                val = special;
            } else {
                int r = bucket_match(q[u], key[u], val);
                // every identifier of the batch is in the table; the bound only guards the loop
                for (uint64_t probes = 0; r < 0 && probes < bmask; ++probes) {
                    bk[u] = (bk[u] + 1) & bmask;
                    r = bucket_match(load_bucket(tab, bk[u]), key[u], val);
                }
                if (r != 1) val = kDeferred;
            }
            if (val != kDeferred) {
                labels[i] = val - off;
                flags[i] = 1;
            }
        }
    }
}

template <typename K>
hipError_t launch_output_direct(const GridView& g, const CoreOut& c, const K* keys_in, const K* skeys,
                                const int32_t* cell_label, void* table, int bits, int key_lo, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    HashSlot<K>* tab = reinterpret_cast<HashSlot<K>*>(table);
    const int64_t slots = (1ll << bits) + 1;
    hash_clear_kernel<K><<<dim3((unsigned)std::min<int64_t>(grid_for(slots), 4096)), dim3(kBlock), 0, st>>>(tab, slots,
                                                                                                      kDeferred);
    hash_build_kernel<K><<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(g, c, skeys, cell_label, tab, bits);
    const int parts = (int)std::max<uint32_t>(1u, g.b.tile_pts / kOutputPart);
    output_direct_kernel<K><<<dim3(g.b.tiles * (uint32_t)parts), dim3(kBlock), 0, st>>>(g.b, keys_in, tab, bits,
                                                                                      key_lo, parts);
    return hipGetLastError();
}
template hipError_t launch_output_direct<uint32_t>(const GridView&, const CoreOut&, const uint32_t*, const uint32_t*,
                                                   const int32_t*, void*, int, int, hipStream_t);
template hipError_t launch_output_direct<uint64_t>(const GridView&, const CoreOut&, const uint64_t*, const uint64_t*,
                                                   const int32_t*, void*, int, int, hipStream_t);

// All-core grids without the hash table (identifiers of two words): their
// points' labels go out through the sort permutation, one thread per grid.
__global__ __launch_bounds__(kBlock) void output_allcore_kernel(GridView gv, CoreOut co,
                                                                const int32_t* __restrict__ cell_label) {
    const int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (c >= (int64_t)*gv.ncell_dev) return;
    const uint32_t st = gv.cell_start[c];
    const uint32_t k = gv.cell_start[c + 1] - st;
    if (co.core_cnt[c] != k) return;  // grids with a non-core point: the border pass
    const Inst& I = cell_inst(gv, c);
    const uint32_t off = (uint32_t)I.off;
    int32_t GD_GLOBAL* __restrict__ labels = as_global(I.labels);
    uint8_t GD_GLOBAL* __restrict__ flags = as_global(I.core);
    const int32_t lab = cell_label[c] - (int32_t)off;
    for (uint32_t s = st; s < st + k; ++s) {
        const uint32_t o = gv.sidx[s] - off;
        labels[o] = lab;
        flags[o] = 1;
    }
}

hipError_t launch_output_allcore(const GridView& g, const CoreOut& c, const int32_t* cell_label, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    output_allcore_kernel<<<dim3(grid_for(g.ncell)), dim3(kBlock), 0, st>>>(g, c, cell_label);
    return hipGetLastError();
}

size_t output_table_bytes(int bits, int key_bytes) {
    return (size_t)((1ll << bits) + 1) * (key_bytes == 4 ? 8 : 16);
}

// Border and noise points of grid c (rows [st, st + k)), one wave.
template <int D, bool kWide>
__device__ __forceinline__ void border_grid(const GridView& gv, const CoreOut& co, const uint64_t* __restrict__ nei_off,
                                            const uint32_t* __restrict__ nei, const int32_t* __restrict__ cell_label,
                                            int64_t c, uint32_t st, uint32_t k, uint32_t* s_start, uint32_t* s_excl,
                                            int32_t* s_lab) {
    const int lane = lane_id();
    const Inst& I = cell_inst(gv, c);
    const uint32_t off = (uint32_t)I.off;  // cluster ids and output slots are local to the instance
    int32_t GD_GLOBAL* __restrict__ labels = as_global(I.labels);
    uint8_t GD_GLOBAL* __restrict__ core_flags = as_global(I.core);
    const int32_t own_label = cell_label[c];
    const uint32_t own_min = co.cell_min_core[c];
    const typename Dist<kWide>::T T = inst_T<kWide>(I);
    const uint64_t own_best = own_min == kNone ? ~0ull : (((uint64_t)own_min << 32) | (uint32_t)own_label);
    const uint64_t e0 = nei_off[c], e1 = nei_off[c + 1];
    const double side = D <= 4 ? (double)I.eps / sqrt((double)I.d) : 0.0;
    const double lim = (double)I.eps * (double)I.eps * (1.0 + 1e-9) + 1.0;
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
                    // a query without a hit scans every core point around it;
                    // a grid of a step or more is dropped when no open query
                    // comes within eps of its cell (low d only, where grids
                    // are large: at d = 7 the test cost more than it saved)
                    if constexpr (D <= 4) {
                        if (worst == ~0ull && cn >= (uint32_t)kWave && !cell_near<D>(gv, cc, open, qx, side, lim))
                            cn = 0;
                    }
                }
            }
            const uint32_t incl = wave_incl_scan(cn);
            const uint32_t tot = __shfl(incl, kWave - 1);
            if (tot == 0) continue;
            s_start[lane] = cs;
            s_excl[lane] = incl - cn;
            s_lab[lane] = lab;
            wave_sync();
            for (uint32_t t0 = 0; t0 < tot; t0 += kWave) {
                const uint32_t t = t0 + lane;
                const bool tv = t < tot;
                int j = 0;
#pragma unroll
                for (int step = 32; step > 0; step >>= 1)
                    if (s_excl[j + step] <= t) j += step;
                const uint32_t q = s_start[j] + (t - s_excl[j]);
                int32_t y[D];
                load_row<D>(co.ccrd, tv ? q : 0u, y);
                const uint64_t cand = tv ? (((uint64_t)co.corig[q] << 32) | (uint32_t)s_lab[j]) : ~0ull;
                uint64_t act = open;
                while (act) {
                    const int qi = ffs64(act);
                    act &= act - 1ull;
                    typename Dist<kWide>::T dd = 0;
#pragma unroll
                    for (int jj = 0; jj < D; ++jj) dd += sqd<kWide>(y[jj], readlane(qx[jj], qi));
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

// Reductions within groups of S lanes (S a power of two up to 64).
template <int S>
__device__ __forceinline__ uint32_t group_incl_scan(uint32_t v) {
    const int sub = lane_id() % S;
#pragma unroll
    for (int o = 1; o < S; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, S);
        if (sub >= o) v += t;
    }
    return v;
}

template <int S>
__device__ __forceinline__ uint64_t group_min_u64(uint64_t v) {
#pragma unroll
    for (int o = S / 2; o > 0; o >>= 1) {
        const uint64_t t = __shfl_xor(v, o, S);
        v = t < v ? t : v;
    }
    return v;
}

// Border and noise points with S lanes per grid (a wave serves 64 / S
// grids side by side): the same search as border_grid, with every scan,
// minimum and broadcast taken within the grid's group of lanes.  Loop
// bounds are uniform within a group, so a group's lanes stay converged
// around every cross-lane step.
template <int D, bool kWide, int S>
__global__ __launch_bounds__(kBlock) void output_group_kernel(GridView gv, CoreOut co,
                                                              const uint64_t* __restrict__ nei_off,
                                                              const uint32_t* __restrict__ nei,
                                                              const int32_t* __restrict__ cell_label) {
    constexpr int G = kWave / S;
    __shared__ uint32_t s_start[kWavesPerBlock][kWave];
    __shared__ uint32_t s_excl[kWavesPerBlock][kWave];
    __shared__ int32_t s_lab[kWavesPerBlock][kWave];
    const int w = wave_id(), lane = lane_id();
    const int grp = lane / S, sub = lane % S, g0 = grp * S;
    const uint64_t gmask = (S == kWave ? ~0ull : ((1ull << S) - 1ull)) << g0;
    const int64_t c = (block_id() * kWavesPerBlock + w) * G + grp;
    if (c >= (int64_t)*gv.ncell_dev) return;
    const uint32_t st = gv.cell_start[c];
    const uint32_t k = gv.cell_start[c + 1] - st;
    if (co.core_cnt[c] == k) return;  // all core: written in input order by the hash pass
    const Inst& I = cell_inst(gv, c);
    const uint32_t off = (uint32_t)I.off;  // cluster ids and output slots are local to the instance
    int32_t GD_GLOBAL* __restrict__ labels = as_global(I.labels);
    uint8_t GD_GLOBAL* __restrict__ core_flags = as_global(I.core);
    const int32_t own_label = cell_label[c];
    const uint32_t own_min = co.cell_min_core[c];
    const typename Dist<kWide>::T T = inst_T<kWide>(I);
    const uint64_t own_best = own_min == kNone ? ~0ull : (((uint64_t)own_min << 32) | (uint32_t)own_label);
    const uint64_t e0 = nei_off[c], e1 = nei_off[c + 1];
    uint32_t* sst = &s_start[w][g0];
    uint32_t* sex = &s_excl[w][g0];
    int32_t* slb = &s_lab[w][g0];
    for (uint32_t qb = 0; qb < k; qb += S) {
        const uint32_t s = st + qb + sub;
        const bool v = qb + sub < k;
        const uint8_t isc = v ? co.core[s] : 1;
        if (v && isc) {
            const uint32_t o = gv.sidx[s] - off;
            labels[o] = own_label - (int32_t)off;
            core_flags[o] = 1;
        }
        const uint64_t open = (ballot(v && !isc) & gmask) >> g0;  // the group's non-core queries
        if (!open) continue;
        int32_t qx[D];
        load_row<D>(gv.crd, v ? s : st, qx);
        uint64_t best = own_best;  // lane i of the group: best candidate of query i
        for (uint64_t e = e0; e < e1; e += S) {
            // largest best among open queries: grids whose smallest core index is not below it cannot help
            const uint64_t worst = ~group_min_u64<S>(((open >> sub) & 1ull) ? ~best : ~0ull);
            const uint32_t worst_idx = (uint32_t)(worst >> 32);
            const uint64_t idx = e + sub;
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
            const uint32_t incl = group_incl_scan<S>(cn);
            const uint32_t tot = __shfl(incl, S - 1, S);
            if (tot == 0) continue;
            sst[sub] = cs;
            sex[sub] = incl - cn;
            slb[sub] = lab;
            wave_sync();
            for (uint32_t t0 = 0; t0 < tot; t0 += S) {
                const uint32_t t = t0 + sub;
                const bool tv = t < tot;
                int j = 0;
#pragma unroll
                for (int step = S / 2; step > 0; step >>= 1)
                    if (sex[j + step] <= t) j += step;
                const uint32_t q = sst[j] + (t - sex[j]);
                int32_t y[D];
                load_row<D>(co.ccrd, tv ? q : 0u, y);
                const uint64_t cand = tv ? (((uint64_t)co.corig[q] << 32) | (uint32_t)slb[j]) : ~0ull;
                uint64_t act = open;
                while (act) {
                    const int qi = ffs64(act);
                    act &= act - 1ull;
                    typename Dist<kWide>::T dd = 0;
#pragma unroll
                    for (int jj = 0; jj < D; ++jj) dd += sqd<kWide>(y[jj], __shfl(qx[jj], qi, S));
                    const bool in = tv && dd <= T;
                    if (ballot(in) & gmask) {
                        const uint64_t m = group_min_u64<S>(in ? cand : ~0ull);
                        if (sub == qi && m < best) best = m;
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

// Each wave checks G grids at once (one lane each) and serves only those
// holding a non-core point (the all-core grids were written in input order
// by output_direct_kernel).  With millions of grids G = 64: a wave per grid
// would spend the kernel dispatching waves that exit at once.  With fewer
// grids G = 1: the grids with non-core points sit together at cluster
// borders, and one wave serving several of them one after another would
// be the kernel's tail.
constexpr int64_t kBorderGroupMinGrids = 1 << 20;

template <int D, int G, bool kWide>
__global__ __launch_bounds__(kBlock) void output_kernel(GridView gv, CoreOut co, const uint64_t* __restrict__ nei_off,
                                                        const uint32_t* __restrict__ nei,
                                                        const int32_t* __restrict__ cell_label) {
    __shared__ uint32_t s_start[kWavesPerBlock][kWave];
    __shared__ uint32_t s_excl[kWavesPerBlock][kWave];
    __shared__ int32_t s_lab[kWavesPerBlock][kWave];
    const int w = wave_id(), lane = lane_id();
    const int64_t c0 = (block_id() * kWavesPerBlock + w) * G;
    const int64_t ncell = *gv.ncell_dev;
    uint32_t st_l = 0, k_l = 0;
    bool need = false;
    if (lane < G && c0 + lane < ncell) {
        st_l = gv.cell_start[c0 + lane];
        k_l = gv.cell_start[c0 + lane + 1] - st_l;
        need = co.core_cnt[c0 + lane] != k_l;
    }
    for (uint64_t todo = ballot(need); todo; todo &= todo - 1ull) {
        const int g = ffs64(todo);
        border_grid<D, kWide>(gv, co, nei_off, nei, cell_label, c0 + g, readlane(st_l, g), readlane(k_l, g),
                              s_start[w], s_excl[w], s_lab[w]);
    }
}

hipError_t launch_output(const GridView& g, const CoreOut& c, const uint64_t* nei_off, const uint32_t* nei,
                         const int32_t* cell_label, bool wide, int lanes, hipStream_t st) {
    if (g.ncell == 0) return hipSuccess;
    const unsigned many = grid_for(g.ncell, kWavesPerBlock * kWave), one = grid_for(g.ncell, kWavesPerBlock);
    if (lanes == 16) {  // four grids per wave, side by side
        const unsigned four = grid_for(g.ncell, kWavesPerBlock * 4);
        if (wide)
            GD_DISPATCH_D(g.D, (output_group_kernel<D, true, 16><<<grid_of(four), dim3(kBlock), 0, st>>>(
                                   g, c, nei_off, nei, cell_label)));
        else
            GD_DISPATCH_D(g.D, (output_group_kernel<D, false, 16><<<grid_of(four), dim3(kBlock), 0, st>>>(
                                   g, c, nei_off, nei, cell_label)));
    } else if (wide) {
        GD_DISPATCH_D(g.D, (output_kernel<D, 1, true><<<grid_of(one), dim3(kBlock), 0, st>>>(g, c, nei_off, nei,
                                                                                          cell_label)));
    } else if (g.ncell >= kBorderGroupMinGrids) {
        GD_DISPATCH_D(g.D, (output_kernel<D, kWave, false><<<grid_of(many), dim3(kBlock), 0, st>>>(g, c, nei_off, nei,
                                                                                                cell_label)));
    } else {
        GD_DISPATCH_D(g.D, (output_kernel<D, 1, false><<<grid_of(one), dim3(kBlock), 0, st>>>(g, c, nei_off, nei,
                                                                                           cell_label)));
    }
    return hipGetLastError();
}

}  // namespace gd
