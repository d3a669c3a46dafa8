// C ABI of the library (include/gritdbscan.h): argument checks, workspace,
// and the launch sequence of Algorithm 6 (with the LDF merge order) for a
// batch of instances; dbscan() is a batch of one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "gritdbscan.h"
#include "launch.hpp"
#include "learned.hpp"
#include "radix.hpp"
#include "rows.hpp"
#include "scan.hpp"

using namespace gd;

namespace {

// Device counters of the optional statistics.
struct StatBlock {
    MergeStats merge[kStatSlots];
    CoreStats core[kStatSlots];
};

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

// The workspace buffers a call grows on demand.
struct Bufs {
    DevBuf arena;   // everything sized by the batch's points and dimension
    DevBuf nei;     // the neighbour lists, sized by their total
    DevBuf table;   // identifier -> label hash table of the output pass
    DevBuf sumbuf;  // CellSummary per grid (learned proposal)
    DevBuf huge;    // queue and device-memory bitmaps for core sets beyond the LDS bitmaps
};

// Pairs with a heavy core set (at least kHeavyCore points, or beyond the LDS
// bitmaps): the queue the merge kernels fill and the bitmaps of the
// workgroups that drain it.
struct HugeMerge {
    HugeQueue q{};
    uint64_t* slabs = nullptr;
    uint32_t words = 0, blocks = 0;
};

enum Phase {
    P_MINMAX, P_KEYS, P_SORT, P_GATHER, P_CELLS, P_TREE, P_NEI_COUNT, P_NEI_FILL,
    P_CORE_MARK, P_CORE_COMPACT, P_LDF, P_MERGE, P_LABELS, P_OUTPUT, P_COUNT
};
static_assert(P_COUNT == GD_PHASE_COUNT, "phase table");
const char* const kPhaseNames[P_COUNT] = {
    "minmax", "keys", "radix_sort", "gather", "cells", "grid_tree", "nei_count", "nei_fill",
    "core_mark", "core_compact", "ldf_order", "merge", "labels", "output"};

// Workspace of dbscan_noalloc: one fixed array per device, never
// allocated or freed by a call.  Host code must not use this name as a
// device address (in host code it names a host-side stand-in): gd_create
// looks the device address up once per device and every call uses that.
static __device__ __align__(256) unsigned char scratch[GD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (= `device`), looked up
// on the first call for that device.  nullptr if the lookup failed.
char* scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) == hipSuccess && ptr)
            g_scratch_ptr[device] = (char*)ptr;
        else
            (void)hipGetLastError();
    }
    return g_scratch_ptr[device];
}

}  // namespace

struct gd_ctx {
    int device = 0;
    std::string err;
    Bufs own;              // the context's workspace (hipMalloc'ed, grown on demand)
    Bufs* cur = &own;      // the workspace of the running call
    // dbscan_noalloc: buffers are carved in order from the device's fixed
    // scratch array instead of being allocated
    char* bump_base = nullptr;
    size_t bump_cap = 0, bump_used = 0;
    char* scratch = nullptr;  // this device's scratch array (hipGetSymbolAddress at gd_create)
    Header* hdr_dev = nullptr;
    Header* hdr_host = nullptr;  // pinned
    StatBlock* stats_dev = nullptr;
    StatBlock* stats_host = nullptr;  // pinned
    Inst* inst_dev = nullptr;
    Inst* inst_host = nullptr;  // pinned
    int inst_cap = 0;
    int64_t ws_limit = 0;
    bool stats = false;
    bool ldf = true;               // LDF order (merge_order 1) or identifier order (0)
    bool bfs = false;              // the BFS order of Algorithm 6 (merge_order 2)
    int nei_mode = 0;              // GD_OPT_NEIGHBOR_MODE: 0 auto, 1 lists, 2 walks
    int64_t approx_delta = 0;      // GD_OPT_APPROX_DELTA (0: exact merging)
    int nei_query = kNeiAuto;      // GD_OPT_NEIGHBOR_QUERY (kNeiAuto for option value 0)
    bool last_walk = false;        // the last eager call walked (no full lists)
    bool last_wide = false;        // the last eager call took 64-bit distances
    gd_stats last{};
    // what the last successful call left in the workspace (for gd_debug_*)
    bool have_last = false;
    int64_t last_n = 0, last_ncell = 0;
    int last_d = 0;
    uint64_t last_nei_total = 0;
    const uint32_t* last_sidx = nullptr;
    const uint32_t* last_cell_start = nullptr;
    const int32_t* last_ck = nullptr;
    int64_t last_ck_stride = 0;
    const uint64_t* last_nei_off = nullptr;
    const uint32_t* last_nei = nullptr;
    const uint8_t* last_core = nullptr;
    const int32_t* last_cell_label = nullptr;
    GridView last_g{};
    CoreOut last_co{};
    int64_t last_max_core = 0;
    bool last_summaries = false;
    // learned proposal
    __half* proposal_dev = nullptr;  // GD_MLP_PARAMS halves
    bool proposal_on = false;
    unsigned long long* counter_dev = nullptr;
    // sync-free runs captured into a HIP graph and replayed
    int graph_mode = 1;              // 0 never, 1 dbscan_batched, 2 every call
    // launch tunables (gd_autotune)
    int tile_pts = kPointTile;       // points per workgroup of the point kernels
    int merge_waves = kWavesPerBlock; // waves per workgroup of the FastMerging kernel
    int grid_lanes = 0;               // GD_OPT_GRID_LANES (0: from the mean list length)
    bool pack_rows = true;            // GD_OPT_PACKED_ROWS
    bool fuse_rows = true;            // single instances: rows written by the sort's last pass
    std::string tuning_file;          // gd_set_tuning_file (empty: none)
    uint64_t generation = 0;         // bumped whenever a buffer is reallocated
    hipStream_t gstream = nullptr;   // capture and replay stream
    hipEvent_t gev = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<int64_t> gsig;       // batch shape the graph was captured for
    uint64_t ggen = 0;
    int last_key_bits = 0;
    bool marking = true;
    // phase timing
    bool timing = false;
    bool events_ok = false;
    hipEvent_t ev[P_COUNT][2] = {};
    bool ran[P_COUNT] = {};
    double phase_ms[P_COUNT] = {};
    hipStream_t st = nullptr;

    void mark(int phase, int which) {
        if (!timing || !events_ok || !marking) return;
        if (hipEventRecord(ev[phase][which], st) == hipSuccess && which == 1) ran[phase] = true;
    }

    int fail(int code, const char* fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
};

namespace {

struct DeviceGuard {
    int prev = -1;
    bool ok = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

#define GD_TRY(call)                                                                                        \
    do {                                                                                                    \
        hipError_t e_ = (call);                                                                             \
        if (e_ != hipSuccess) return ctx->fail(GD_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Bump allocator over one device buffer.
struct Carve {
    char* base;
    size_t off = 0;
    template <typename T>
    T* take(int64_t count) {
        T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
        off += align_up((size_t)std::max<int64_t>(count, 1) * sizeof(T));
        return p;
    }
};

int grow(gd_ctx* ctx, DevBuf& b, size_t need, size_t other_held) {
    if (need <= b.cap) return GD_OK;
    if (ctx->bump_base) {
        // no allocation: the next slice of the fixed scratch array
        const size_t off = align_up(ctx->bump_used);
        if (off > ctx->bump_cap || need > ctx->bump_cap - off)
            return ctx->fail(GD_ENOMEM,
                             "dbscan_noalloc: the call needs more than the fixed %llu-byte scratch "
                             "(%zu bytes already taken, %zu more asked)",
                             (unsigned long long)ctx->bump_cap, off, need);
        b.p = ctx->bump_base + off;
        b.cap = need;
        ctx->bump_used = off + need;
        return GD_OK;
    }
    if (ctx->ws_limit > 0 && (int64_t)(need + other_held) > ctx->ws_limit)
        return ctx->fail(GD_ENOMEM, "workspace of %zu bytes exceeds the context limit of %lld bytes", need + other_held,
                         (long long)ctx->ws_limit);
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
    }
    const size_t sz = need + need / 8;  // some headroom for the next call
    ++ctx->generation;                  // a captured graph that used the old buffer is stale
    if (hipMalloc(&b.p, sz) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return ctx->fail(GD_ENOMEM, "hipMalloc of %zu bytes failed", sz);
    }
    b.cap = sz;
    return GD_OK;
}

int bit_length(uint64_t v) { return v == 0 ? 0 : 64 - __builtin_clzll(v); }

// Capacities of a sync-free run (see run_batch).
struct Plan {
    int key_bits;      // identifier bits sorted (a multiple of 8)
    int64_t ncell;     // grids
    uint64_t nei;      // neighbour-list entries
    int64_t ncc;       // core grids
    int64_t max_core;  // largest core set
    bool walk;         // consumers walk the grid tree (lists only for big core sets)
};

// Largest delta of approximate merging: (eps + delta)^2 must fit 32 bits.
constexpr int kApproxDeltaMax = 65535 - GD_EPS_MAX;
constexpr int64_t kEpsClamp = (int64_t)1 << 27;

// build_lists: the full lists do not fit the workspace (limit or fixed
// scratch) and the consumers may walk the grid tree instead.
constexpr int kListsDoNotFit = 1;

// Hash tables of the grids (the hashing neighbour query's, the output's):
// 2^bits slots for ncell grids, load <= 1/8 up to 2^20 grids (fewer second
// probes), <= 1/4 above (the table stays modest).  A planned run's table
// buffer is sized by this bound, which covers both.
int table_bits(int64_t ncell) {
    const int64_t slots = ncell <= (1 << 20) ? 8 * ncell : 4 * ncell;
    int b = 10;
    while (((int64_t)1 << b) < slots) ++b;
    return b;
}

// The output table holds only the all-core grids, and above 2^20 grids it is
// cleared in every call: 2 slots per grid there (load <= 1/2, in practice
// the all-core share of that) halves the clearing of a table that outgrows
// the caches anyway.
int output_table_bits(int64_t ncell) {
    if (ncell <= (1 << 20)) return table_bits(ncell);
    int b = 10;
    while (((int64_t)1 << b) < 2 * ncell) ++b;
    return b;
}

// Workspace layout; with base == nullptr it only measures.
struct Layout {
    uint32_t* vals_a;
    uint32_t* vals_b;
    void* keys_a;
    void* keys_b;
    void* keys_c;
    uint32_t* radix_scratch;
    uint64_t* partial;
    int32_t* crd;
    uint32_t* cell_start;
    int32_t* ck;
    uint32_t* level_excl;
    int32_t* tkey[kMaxLevels];
    uint32_t* tchild[kMaxLevels];
    uint32_t* off_counts;
    uint2* nei_up;
    uint64_t* nei_off;
    uint8_t* core;
    uint32_t* core_cnt;
    uint32_t* core_begin;
    uint32_t* side_off;
    uint32_t* count_part;
    uint32_t* cell_min_core;
    int32_t* tile_mm;
    uint32_t* list;
    uint4* rank;
    uint32_t* parent;
    uint32_t* root_min;
    int32_t* cell_label;
    size_t bytes;
};

// Bytes of a packed identifier of `bits` bits: one 32- or 64-bit word, or two.
int key_bytes_of(int bits) { return bits <= 32 ? 4 : bits <= 64 ? 8 : 16; }

Layout carve(char* base, int64_t n, int D, uint32_t tiles, int key_bytes = 8) {
    Layout L{};
    Carve c{base};
    const int64_t kw = std::max(key_bytes, 8) / 8;  // identifier buffers hold n 64-bit words, or 2n
    L.keys_a = c.take<uint64_t>(kw * n);  // identifiers in input order (kept for the output pass)
    L.keys_b = c.take<uint64_t>(kw * n);
    L.keys_c = c.take<uint64_t>(kw * n);
    // the sorted index doubles as the row -> input index map of the core
    // sets, whose side area follows row n
    L.vals_a = c.take<uint32_t>(2 * n);
    L.vals_b = c.take<uint32_t>(2 * n);
    const int64_t big_scan = std::max<int64_t>(n + 1, (int64_t)radix_max_bins<uint32_t>() * radix_tiles(n));
    L.radix_scratch = c.take<uint32_t>(radix_scratch_words(n));
    L.partial = c.take<uint64_t>(scan_partial_cap(big_scan) + 4);
    L.crd = c.take<int32_t>((int64_t)row_stride(D) * 2 * n);  // sorted rows, then the side area
    L.cell_start = c.take<uint32_t>(n + 1);
    L.ck = c.take<int32_t>((int64_t)(D + 1) * n);
    L.level_excl = c.take<uint32_t>((int64_t)D * (n + 1));
    for (int l = 0; l < D; ++l) {
        L.tkey[l] = c.take<int32_t>(n);
        L.tchild[l] = c.take<uint32_t>(n + 1);
    }
    L.off_counts = c.take<uint32_t>((int64_t)D * n);
    L.nei_off = c.take<uint64_t>(n + 1);
    L.nei_up = c.take<uint2>(n);
    L.core = c.take<uint8_t>(n);
    L.core_cnt = c.take<uint32_t>(n);
    L.core_begin = c.take<uint32_t>(n);
    L.side_off = c.take<uint32_t>(n + 1);
    L.count_part = c.take<uint32_t>(5 * (n / kBlock + 2));
    L.cell_min_core = c.take<uint32_t>(n);
    L.tile_mm = c.take<int32_t>((int64_t)2 * kMaxD * tiles);
    L.list = c.take<uint32_t>(n);
    L.rank = c.take<uint4>(n);
    L.parent = c.take<uint32_t>(n);
    L.root_min = c.take<uint32_t>(n);
    L.cell_label = c.take<int32_t>(n);
    L.bytes = c.off;
    return L;
}

int readback(gd_ctx* ctx, hipStream_t st) {
    GD_TRY(hipMemcpyAsync(ctx->hdr_host, ctx->hdr_dev, sizeof(Header), hipMemcpyDeviceToHost, st));
    GD_TRY(hipStreamSynchronize(st));
    return GD_OK;
}

// The identifier sort of one instance with packed rows, its last pass
// writing the sorted rows, index and identifiers (PackedRowsOut).
hipError_t sort_packed_rows(const Batch& b, uint32_t* ka, uint64_t* va, uint32_t* kb, uint64_t* vb, int key_bits,
                            const Layout& L, hipStream_t st, RadixResult<uint32_t, uint64_t>* r) {
    GD_DISPATCH_D(b.D, ({
                      PackedRowsOut<D> o{};
                      o.inst = b.inst;
                      o.crd = L.crd;
                      return radix_sort_pairs<uint32_t, uint64_t, PackedRowsOut<D>>(
                          ka, va, kb, vb, b.n, key_bits, false, L.radix_scratch, st, r,
                          reinterpret_cast<uint32_t*>(L.keys_c), 0, &o);
                  }));
    return hipErrorInvalidValue;
}

// Bits per coordinate that every instance's grids fit (pack64_bits), 0 if
// some instance's do not fit 31 bits.
int pack64_width(const gd_ctx* ctx, int count) {
    int bits = 0;
    for (int k = 0; k < count; ++k) {
        const int bk = pack64_bits(ctx->inst_host[k].d, ctx->inst_host[k].eps);
        if (bk == 0) return 0;
        bits = std::max(bits, bk);
    }
    return bits;
}

template <typename K>
int run_partition(gd_ctx* ctx, const Batch& b, int key_bits, Layout& L, const uint32_t** sidx_out, void** skeys_out,
                  int* key_lo_out, hipStream_t st) {
    K* ka = (K*)L.keys_a;
    K* kb = (K*)L.keys_b;
    *key_lo_out = 0;
    // With 32-bit identifiers and every instance's grid side small enough,
    // the sort carries each point's low coordinate bits and the sorted rows
    // are rebuilt in sorted order (no random gather).  The value buffers
    // hold 2n u32 each, so n u64 values fit.
    bool pack = std::is_same<K, uint32_t>::value && ctx->pack_rows;
    for (int k = 0; k < b.count && pack; ++k) pack = pack_fits(ctx->inst_host[k].d, ctx->inst_host[k].eps);
    // Two-word keys: the low coordinate bits ride in the key word itself,
    // below the identifier, when both fit in 64 bits (B bits per coordinate
    // for the whole batch); the sort orders on the identifier bits only.
    int pack64_b = 0;
    if (std::is_same<K, uint64_t>::value && ctx->pack_rows) {
        pack64_b = pack64_width(ctx, b.count);
        if (pack64_b > 0 && key_bits + b.D * pack64_b > 64) pack64_b = 0;
    }
    RadixResult<K> res;
    if (pack64_b > 0) {
        const int W = b.D * pack64_b;
        uint64_t* wa = reinterpret_cast<uint64_t*>(ka);
        ctx->mark(P_KEYS, 0);
        GD_TRY(launch_keys_packed64(b, wa, pack64_b, st));
        ctx->mark(P_KEYS, 1);
        RadixResult<uint64_t> rw;
        ctx->mark(P_SORT, 0);
        GD_TRY((radix_sort_pairs<uint64_t>(wa, L.vals_a, reinterpret_cast<uint64_t*>(kb), L.vals_b, b.n, key_bits, true,
                                           L.radix_scratch, st, &rw, reinterpret_cast<uint64_t*>(L.keys_c), W)));
        ctx->mark(P_SORT, 1);
        ctx->mark(P_GATHER, 0);
        GD_TRY(launch_unpack64(b, rw.keys, pack64_b, L.crd, st));
        ctx->mark(P_GATHER, 1);
        res.keys = reinterpret_cast<K*>(rw.keys);
        res.vals = rw.vals;
        *key_lo_out = W;
    } else if (pack) {
        uint64_t* va = reinterpret_cast<uint64_t*>(L.vals_a);
        uint64_t* vb = reinterpret_cast<uint64_t*>(L.vals_b);
        ctx->mark(P_KEYS, 0);
        GD_TRY(launch_keys<K>(b, ka, va, st));
        ctx->mark(P_KEYS, 1);
        RadixResult<K, uint64_t> r64{};
        ctx->mark(P_SORT, 0);
        if constexpr (std::is_same<K, uint32_t>::value) {
            if (b.count == 1 && ctx->fuse_rows)
                // one instance: the last pass writes the rows, the index and
                // the identifiers itself
                GD_TRY(sort_packed_rows(b, ka, va, kb, vb, key_bits, L, st, &r64));
            else
                GD_TRY((radix_sort_pairs<K, uint64_t>(ka, va, kb, vb, b.n, key_bits, false, L.radix_scratch, st,
                                                      &r64, (K*)L.keys_c)));
        }
        ctx->mark(P_SORT, 1);
        if (r64.last_fused) {
            res.keys = r64.keys;
            res.vals = reinterpret_cast<uint32_t*>(r64.vals);
        } else {
            // sidx goes to the value buffer the sorted values are not in
            uint32_t* sidx = r64.vals == va ? L.vals_b : L.vals_a;
            ctx->mark(P_GATHER, 0);
            GD_TRY(launch_unpack(b, reinterpret_cast<const uint32_t*>(r64.keys), r64.vals, sidx, L.crd, st));
            ctx->mark(P_GATHER, 1);
            res.keys = r64.keys;
            res.vals = sidx;
        }
    } else {
        ctx->mark(P_KEYS, 0);
        GD_TRY(launch_keys<K>(b, ka, nullptr, st));
        ctx->mark(P_KEYS, 1);
        ctx->mark(P_SORT, 0);
        GD_TRY(radix_sort_pairs<K>(ka, L.vals_a, kb, L.vals_b, b.n, key_bits, true, L.radix_scratch, st, &res,
                                   (K*)L.keys_c));
        ctx->mark(P_SORT, 1);
        ctx->mark(P_GATHER, 0);
        GD_TRY(launch_gather(b, res.vals, L.crd, st));
        ctx->mark(P_GATHER, 1);
    }
    ctx->mark(P_CELLS, 0);
    GD_TRY(launch_cells<K>(b, res.keys, (uint32_t*)L.partial, L.cell_start, L.ck, b.n, st));
    ctx->mark(P_CELLS, 1);
    *sidx_out = res.vals;
    *skeys_out = res.keys;
    return GD_OK;
}

// The merge in the BFS order of Algorithm 6: rounds of seeds, each
// followed by breadth-first levels until the frontier is empty; every level
// reads its frontier size back (an eager run only).
int run_bfs(gd_ctx* ctx, const GridView& g, const CoreOut& co, const uint64_t* nei_off, const uint32_t* nei,
            int64_t max_core, const HugeMerge& hm, bool wide, uint32_t* state, uint32_t* front, uint32_t* next,
            uint32_t* cnt, uint32_t* parent, MergeStats* stats, hipStream_t st) {
    GD_TRY(fill<uint32_t>(state, g.ncell, 0u, st));
    uint32_t h[3];
    for (;;) {
        GD_TRY(fill<uint32_t>(cnt, 3, 0u, st));
        GD_TRY(launch_bfs_seeds(g, co, nei_off, nei, state, front, cnt, st));
        GD_TRY(hipMemcpyAsync(h, cnt, sizeof(h), hipMemcpyDeviceToHost, st));
        GD_TRY(hipStreamSynchronize(st));
        if (h[0] == 0) return GD_OK;  // every core grid is classified
        uint32_t nf = h[1];
        while (nf > 0) {
            GD_TRY(fill<uint32_t>(cnt + 2, 1, 0u, st));
            if (hm.q.pairs) GD_TRY(fill<uint32_t>(hm.q.count, 1, 0u, st));
            GD_TRY(launch_bfs_level(g, co, nei_off, nei, front, nf, next, cnt, max_core, hm.q, wide, state, parent,
                                    stats, st));
            GD_TRY(launch_merge_huge(g, co, hm.q, hm.slabs, hm.words, hm.blocks, true, wide, state, next, cnt, parent,
                                     stats, st));
            GD_TRY(hipMemcpyAsync(h + 2, cnt + 2, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
            GD_TRY(hipStreamSynchronize(st));
            nf = h[2];
            std::swap(front, next);
        }
    }
}

// Validated batch in ctx->inst_host[0..count): run every phase.  With a
// plan the run is sync-free (every buffer already grown, capacities from
// the plan, no host readback until the end) so that it can be captured into
// a HIP graph; device-side checks raise kErrPlan when the data outgrow it.
int run_batch(gd_ctx* ctx, int count, int D, int64_t n, uint32_t tiles, hipStream_t st, const Plan* plan) {
    ctx->have_last = false;
    std::memset(&ctx->last, 0, sizeof(ctx->last));
    ctx->last.n = n;
    ctx->last.d = D;
    if (n == 0) return GD_OK;

    // ---- workspace (identifiers of one word; two once the layout needs them)
    int kbytes = plan ? key_bytes_of(plan->key_bits) : 8;
    Layout L = carve(nullptr, n, D, tiles, kbytes);
    int rc = plan ? GD_OK : grow(ctx, ctx->cur->arena, L.bytes, ctx->cur->nei.cap);
    if (rc) return rc;
    L = carve((char*)ctx->cur->arena.p, n, D, tiles, kbytes);
    Header* Hd = ctx->hdr_dev;
    Header* H = ctx->hdr_host;

    Batch b{};
    b.inst = ctx->inst_dev;
    b.count = count;
    b.D = D;
    b.n = n;
    b.tiles = tiles;
    b.tile_pts = (uint32_t)ctx->tile_pts;
    b.hdr = Hd;

    ctx->st = st;
    ctx->marking = !plan;
    for (int p = 0; p < P_COUNT; ++p) {
        ctx->ran[p] = false;
        ctx->phase_ms[p] = 0.0;
    }

    // ---- instance table, mn_j and the input check (Eq. (1)), identifier layout
    GD_TRY(hipMemcpyAsync(ctx->inst_dev, ctx->inst_host, sizeof(Inst) * count, hipMemcpyHostToDevice, st));
    GD_TRY(fill<uint32_t>((uint32_t*)Hd, (int64_t)(sizeof(Header) / sizeof(uint32_t)), 0u, st));
    const bool stats = ctx->stats && !plan;
    if (stats)
        GD_TRY(fill<unsigned long long>(&ctx->stats_dev->merge[0].pairs,
                                        (int64_t)(sizeof(StatBlock) / sizeof(unsigned long long)), 0ull, st));
    ctx->mark(P_MINMAX, 0);
    GD_TRY(launch_minmax(b, L.tile_mm, plan ? plan->key_bits : kMaxKeyBits, st));
    ctx->mark(P_MINMAX, 1);
    if (!plan && (rc = readback(ctx, st))) return rc;
    if (!plan && (H->err & kErrNotInteger)) {
        GD_TRY(hipMemcpyAsync(ctx->inst_host, ctx->inst_dev, sizeof(Inst) * count, hipMemcpyDeviceToHost, st));
        GD_TRY(hipStreamSynchronize(st));
        int bad = 0;
        while (bad < count && !(ctx->inst_host[bad].err & kErrNotInteger)) ++bad;
        return ctx->fail(GD_ERANGE, "instance %d: a coordinate is not a finite integer of magnitude <= 2^24", bad);
    }
    if (!plan && (H->err & kErrKeyBits))
        return ctx->fail(GD_ERANGE, "grid identifiers need %d bits (> %d): eps too small for the data's extent",
                         H->total_bits, kMaxKeyBits);
    const int key_bits = plan ? plan->key_bits : H->total_bits;
    ctx->last.key_bits = key_bits;
    if (key_bytes_of(key_bits) > kbytes) {
        // two-word identifiers: the identifier buffers double (the min/max
        // records, the only data so far, are folded into the instance table)
        kbytes = key_bytes_of(key_bits);
        if ((rc = grow(ctx, ctx->cur->arena, carve(nullptr, n, D, tiles, kbytes).bytes, ctx->cur->nei.cap))) return rc;
        L = carve((char*)ctx->cur->arena.p, n, D, tiles, kbytes);
    }
    // the narrowest word that holds the identifiers (32-bit identifiers sort
    // and carry packed rows as one-word keys; the buffers carved for a wider
    // word hold them too)
    kbytes = key_bytes_of(key_bits);
    if (kbytes > 8 && ctx->nei_query == kNeiHash)
        return ctx->fail(GD_EUNSUPPORTED, "the hashing neighbour query takes identifiers of at most 64 bits (%d here)",
                         key_bits);

    // ---- Algorithm 1: identifiers, radix sort, grids
    const uint32_t* sidx = nullptr;
    void* skeys = nullptr;
    int key_lo = 0;  // bits below the identifier in the input-order key words
    // 32-bit identifiers whose grids are too wide for the packed value
    // (pack_fits) sort as 64-bit words with the rows packed below them when
    // both fit: a third more bytes per sort pass instead of a random gather
    if (kbytes == 4 && ctx->pack_rows) {
        bool fits32 = true;
        for (int k = 0; k < count && fits32; ++k) fits32 = pack_fits(ctx->inst_host[k].d, ctx->inst_host[k].eps);
        const int pb = fits32 ? 0 : pack64_width(ctx, count);
        if (pb > 0 && key_bits + D * pb <= 64) kbytes = 8;
    }
    if (kbytes == 4)
        rc = run_partition<uint32_t>(ctx, b, key_bits, L, &sidx, &skeys, &key_lo, st);
    else if (kbytes == 8)
        rc = run_partition<uint64_t>(ctx, b, key_bits, L, &sidx, &skeys, &key_lo, st);
    else
        rc = run_partition<Key128>(ctx, b, key_bits, L, &sidx, &skeys, &key_lo, st);
    if (rc) return rc;
    if (plan)
        GD_TRY(launch_plan_check(Hd, 0, plan->ncell, 0, st));
    else if ((rc = readback(ctx, st)))
        return rc;
    const int64_t ncell = plan ? plan->ncell : (int64_t)H->ncell;

    GridView g{};
    g.b = b;
    g.n = n;
    g.D = D;
    g.crd = L.crd;
    g.sidx = sidx;
    g.ncell = ncell;
    g.ncell_dev = &Hd->ncell;
    g.cell_start = L.cell_start;
    g.ck = L.ck;
    g.ck_stride = n;

    // ---- Algorithm 2 (grid tree) and Algorithm 3 (Nei for every grid)
    ctx->mark(P_TREE, 0);
    GD_TRY(launch_tree(g, L.level_excl, (uint32_t*)L.partial, L.tkey, L.tchild, st));
    ctx->mark(P_TREE, 1);
    TreeView t{};
    for (int l = 0; l < D; ++l) {
        t.key[l] = L.tkey[l];
        t.child[l] = L.tchild[l];
    }
    t.key[D] = L.ck + (int64_t)D * n;
    t.level_count = Hd->level_count;
    // Lists for every grid, unless asked to walk (the BFS order expands
    // every core grid over its full list) or, by default, when the lists do
    // not fit the workspace: then the consumers walk the grid tree.
    bool walk = plan ? plan->walk : (!ctx->bfs && ctx->nei_mode == 2);
    const bool may_walk = !plan && !ctx->bfs && ctx->nei_mode == 0;
    // the split walk's per-lane counts go to the sort buffer that does not
    // hold the sorted identifiers (free until the LDF step), when they fit
    uint64_t nei_total = 0;
    uint32_t* nei = nullptr;
    bool lists_up = false;  // L.nei_up holds each list's larger-index range
    // Nei(g) of every grid, or (walk mode) of the grids with more than
    // kTinyCore core points, known only after core marking
    auto build_lists = [&](const uint32_t* only_big, bool fallback) -> int {
        NeiQuery nq{};
        nq.t = t;
        // offset order pays for itself through core marking's early exit
        // only when grids hold several points; sparse grids take walk order,
        // and so do more than 2^19 grids, whose ordered fill (scattered over
        // the offset buckets) outweighs the early exit
        int kind = ctx->nei_query;
        if (kind == kNeiAuto)
            kind = ncell <= ((int64_t)1 << 19) && n >= 8 * std::max<int64_t>(ncell, 1) ? kNeiTree : kNeiTreeWalkOrder;
        nq.kind = only_big ? kNeiTree : kind;
        nq.key_bytes = kbytes;
        nq.inst = b.inst;
        nq.inst_shift = &Hd->inst_shift;
        // the split query's per-lane counts go to the sort buffer that does
        // not hold the sorted identifiers (free until the LDF step), when
        // they fit
        uint32_t* lane_cnt = nullptr;
        const int64_t words = nei_lane_count_words(nq, ncell, D);
        if (words > 0 && words <= 2 * n) lane_cnt = (uint32_t*)(skeys == L.keys_b ? L.keys_c : L.keys_b);
        ctx->mark(P_NEI_COUNT, 0);
        if (nq.kind == kNeiHash) {
            // the identifier -> grid table lives in the output pass's table
            // buffer, which that pass clears and refills later
            nq.bits = table_bits(ncell);
            int rc2;
            if (!plan && (rc2 = grow(ctx, ctx->cur->table, output_table_bytes(nq.bits, nq.key_bytes),
                                     ctx->cur->arena.cap)))
                return rc2;
            nq.table = ctx->cur->table.p;
            GD_TRY(launch_grid_table(g, skeys, nq.key_bytes, ctx->cur->table.p, nq.bits, st));
        }
        GD_TRY(launch_nei_count(g, nq, L.off_counts, lane_cnt, only_big, st));
        GD_TRY(launch_nei_offsets(g, L.off_counts, L.nei_off, L.partial, st));
        ctx->mark(P_NEI_COUNT, 1);
        int rc2;
        if (plan)
            GD_TRY(launch_plan_check(Hd, 1, (int64_t)plan->nei, 0, st));
        else if ((rc2 = readback(ctx, st)))
            return rc2;
        nei_total = plan ? plan->nei : H->nei_total;
        if (!plan && (rc2 = grow(ctx, ctx->cur->nei, (size_t)std::max<uint64_t>(nei_total, 1) * sizeof(uint32_t),
                                 ctx->cur->arena.cap))) {
            if (fallback && rc2 == GD_ENOMEM) {
                ctx->err.clear();
                return kListsDoNotFit;
            }
            return rc2;
        }
        nei = (uint32_t*)ctx->cur->nei.p;
        ctx->mark(P_NEI_FILL, 0);
        GD_TRY(launch_nei_fill(g, nq, L.off_counts, lane_cnt, L.nei_off, nei, nei_total, only_big, L.nei_up, st));
        lists_up = nei_walk_order(nq, ncell);
        ctx->mark(P_NEI_FILL, 1);
        return GD_OK;
    };
    if (!walk) {
        rc = build_lists(nullptr, may_walk);
        if (rc == kListsDoNotFit)
            walk = true;
        else if (rc)
            return rc;
    }
    ctx->last.neighbor_walk = walk ? 1 : 0;
    // lanes per grid in the kernels that serve small grids (tiny-set merge,
    // border points): short lists leave most of a wave per grid idle
    const uint64_t grids = (uint64_t)std::max<int64_t>(ncell, 1);
    const int small_lanes =
        ctx->grid_lanes ? ctx->grid_lanes : (nei_total <= 40 * grids && (uint64_t)n <= 32 * grids ? 16 : 64);

    // ---- core points
    ctx->mark(P_CORE_MARK, 0);
    int64_t max_eps = 0, min_minpts = INT64_MAX;
    for (int k = 0; k < count; ++k) {
        max_eps = std::max<int64_t>(max_eps, ctx->inst_host[k].eps);
        min_minpts = std::min<int64_t>(min_minpts, ctx->inst_host[k].minpts);
    }
    // eps above the 32-bit bound anywhere in the batch: 64-bit distances
    const bool wide = max_eps > GD_EPS_MAX;
    if (walk)
        GD_TRY(launch_core_walk(g, t, L.core, L.core_cnt, stats ? ctx->stats_dev->core : nullptr, wide, st));
    else
        GD_TRY(launch_core_mark(g, L.nei_off, nei, L.core, L.core_cnt, stats ? ctx->stats_dev->core : nullptr,
                                max_eps, min_minpts, n >= 1024 * std::max<int64_t>(ncell, 1), st));
    ctx->mark(P_CORE_MARK, 1);
    CoreOut co{};
    co.core = L.core;
    co.core_cnt = L.core_cnt;
    co.core_begin = L.core_begin;
    co.ccrd = L.crd;
    co.corig = const_cast<uint32_t*>(sidx);
    co.side_off = L.side_off;
    co.count_part = L.count_part;
    co.cell_min_core = L.cell_min_core;
    co.counts = Hd->counts;
    ctx->mark(P_CORE_COMPACT, 0);
    GD_TRY(launch_core_compact(g, co, (uint32_t*)L.partial, st));
    ctx->mark(P_CORE_COMPACT, 1);
    if (plan)
        GD_TRY(launch_plan_check(Hd, 2, plan->ncc, plan->max_core, st));
    else if ((rc = readback(ctx, st)))
        return rc;
    const int64_t ncore = plan ? 0 : (int64_t)H->counts[0];
    const int64_t ncc = plan ? plan->ncc : (int64_t)H->counts[1];
    const int64_t max_core = plan ? plan->max_core : (int64_t)H->counts[2];
    if (walk && (rc = build_lists(L.core_cnt, false))) return rc;
    // heavy core sets: their pairs are queued and merged by whole workgroups
    // (never in a planned run: a replay tests them on one wave each, and one
    // that meets a set beyond the LDS bitmaps runs again eagerly)
    HugeMerge hm;
    if (!plan && max_core >= kHeavyCore) {
        unsigned long long lists = 0;
        GD_TRY(fill<unsigned long long>(ctx->counter_dev, 1, 0ull, st));
        GD_TRY(launch_huge_scan(g, co, L.nei_off, ctx->counter_dev, st));
        GD_TRY(hipMemcpyAsync(&lists, ctx->counter_dev, sizeof(lists), hipMemcpyDeviceToHost, st));
        GD_TRY(hipStreamSynchronize(st));
        const uint64_t cap = 2 * (uint64_t)lists + 64;
        if (cap > 0xffffffffull)
            return ctx->fail(GD_EUNSUPPORTED, "%llu neighbour pairs of heavy core sets", (unsigned long long)cap);
        hm.words = (uint32_t)((max_core + kWave - 1) / kWave);
        const size_t slab = (size_t)2 * hm.words * sizeof(uint64_t);
        // as many workgroups as pairs, up to 512 and 256 MiB of bitmaps
        hm.blocks = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(cap, 512),
                                                 std::max<size_t>((256u << 20) / slab, 1));
        const size_t qbytes = align_up(cap * sizeof(uint2) + sizeof(uint32_t));
        if ((rc = grow(ctx, ctx->cur->huge, qbytes + (size_t)hm.blocks * slab,
                       ctx->cur->arena.cap + ctx->cur->nei.cap + ctx->cur->table.cap + ctx->cur->sumbuf.cap)))
            return rc;
        char* b = (char*)ctx->cur->huge.p;
        hm.q.pairs = (uint2*)b;
        hm.q.cap = (uint32_t)cap;
        hm.q.count = (uint32_t*)(b + cap * sizeof(uint2));
        hm.slabs = (uint64_t*)(b + qbytes);
        GD_TRY(fill<uint32_t>(hm.q.count, 1, 0u, st));
    }

    // ---- merging (Algorithm 5 + union-find, LDF order)
    uint32_t* ldf = nullptr;
    {
        // the sort buffer that does not hold the sorted identifiers is free
        uint32_t* ka = (uint32_t*)(skeys == L.keys_b ? L.keys_c : L.keys_b);
        uint32_t* kb = ka + n;
        uint32_t* vb = (sidx == L.vals_a) ? L.vals_b : L.vals_a;
        ctx->mark(P_LDF, 0);
        // a planned run sorts ncc slots, the unused ones last under an all-ones key
        const int count_bits = bit_length((uint64_t)max_core) + (plan ? 1 : 0);
        GD_TRY(launch_ldf_order(g, co, ctx->ldf && !ctx->bfs, ncc, count_bits, plan != nullptr, L.list, L.rank,
                                L.parent, L.root_min, ka, kb, vb, L.radix_scratch, (uint32_t*)L.partial, &ldf, st));
        ctx->mark(P_LDF, 1);
        if (ctx->bfs && !plan) {
            // Algorithm 6's order: the free sort buffers hold the grid states
            // and the two frontiers, the radix scratch the counters
            ctx->mark(P_MERGE, 0);
            rc = run_bfs(ctx, g, co, L.nei_off, nei, max_core, hm, wide, ka, kb, vb, L.radix_scratch, L.parent,
                         stats ? ctx->stats_dev->merge : nullptr, st);
            if (rc) return rc;
            ctx->mark(P_MERGE, 1);
        }
    }
    CellSummary* sum = nullptr;
    ctx->last_summaries = false;
    if (ctx->proposal_on) {
        if (!plan && (rc = grow(ctx, ctx->cur->sumbuf, sizeof(CellSummary) * (size_t)std::max<int64_t>(ncell, 1),
                                ctx->cur->arena.cap + ctx->cur->nei.cap)))
            return rc;
        sum = (CellSummary*)ctx->cur->sumbuf.p;
    }
    if (!ctx->bfs || plan) {
        ctx->mark(P_MERGE, 0);
        if (sum) {
            GD_TRY(launch_summaries(g, co, sum, st));
            ctx->last_summaries = true;
        }
        const int64_t n_small = !ctx->ldf ? -1 : plan ? -2 : (int64_t)H->counts[4];
        if (walk)
            GD_TRY(launch_merge_walk(g, co, t, ldf, n_small, L.parent, stats ? ctx->stats_dev->merge : nullptr, wide,
                                     st));
        GD_TRY(launch_merge(g, co, L.nei_off, nei, lists_up && !walk ? L.nei_up : nullptr, ldf, L.rank, ncc,
                            n_small, max_core, ctx->merge_waves,
                            small_lanes, walk,
                            hm.q, wide, L.parent, stats ? ctx->stats_dev->merge : nullptr,
                            ctx->proposal_on ? ctx->proposal_dev : nullptr, sum, st));
        GD_TRY(launch_merge_huge(g, co, hm.q, hm.slabs, hm.words, hm.blocks, false, wide, nullptr, nullptr, nullptr,
                                 L.parent, stats ? ctx->stats_dev->merge : nullptr, st));
        ctx->mark(P_MERGE, 1);
    }
    ctx->mark(P_LABELS, 0);
    GD_TRY(launch_labels(g, co, L.parent, L.root_min, L.cell_label, st));
    ctx->mark(P_LABELS, 1);

    // ---- border / noise, output in input order
    const int hbits = output_table_bits(ncell);
    if (!plan && kbytes <= 8 &&
        (rc = grow(ctx, ctx->cur->table, output_table_bytes(hbits, kbytes),
                   ctx->cur->arena.cap + ctx->cur->nei.cap + ctx->cur->sumbuf.cap + ctx->cur->huge.cap)))
        return rc;
    ctx->mark(P_OUTPUT, 0);
    if (kbytes == 4)
        GD_TRY(launch_output_direct<uint32_t>(g, co, (const uint32_t*)L.keys_a, (const uint32_t*)skeys, L.cell_label,
                                              ctx->cur->table.p, hbits, 0, st));
    else if (kbytes == 8)
        GD_TRY(launch_output_direct<uint64_t>(g, co, (const uint64_t*)L.keys_a, (const uint64_t*)skeys, L.cell_label,
                                              ctx->cur->table.p, hbits, key_lo, st));
    else
        GD_TRY(launch_output_allcore(g, co, L.cell_label, st));
    if (walk)
        GD_TRY(launch_border_walk(g, co, t, L.cell_label, wide, st));
    else
        GD_TRY(launch_output(g, co, L.nei_off, nei, L.cell_label, wide, small_lanes, st));
    ctx->mark(P_OUTPUT, 1);
    if (stats) GD_TRY(hipMemcpyAsync(ctx->stats_host, ctx->stats_dev, sizeof(StatBlock), hipMemcpyDeviceToHost, st));
    if (plan) {
        // the caller synchronises and checks the header
        GD_TRY(hipMemcpyAsync(ctx->hdr_host, ctx->hdr_dev, sizeof(Header), hipMemcpyDeviceToHost, st));
        return GD_OK;
    }
    if ((rc = readback(ctx, st))) return rc;
    if (H->err & kErrMergeRunaway) return ctx->fail(GD_EDEVICE, "merge step exceeded its iteration bound");
    if (H->err & (kErrNeiOverflow | kErrCoreCap))
        return ctx->fail(GD_EDEVICE, "internal capacity check failed (error bits 0x%x)", H->err);
    if (ctx->timing && ctx->events_ok) {
        for (int p = 0; p < P_COUNT; ++p) {
            float ms = 0.f;
            if (ctx->ran[p] && hipEventElapsedTime(&ms, ctx->ev[p][0], ctx->ev[p][1]) == hipSuccess)
                ctx->phase_ms[p] = ms;
        }
    }

    ctx->have_last = true;
    ctx->last_n = n;
    ctx->last_d = D;
    ctx->last_ncell = ncell;
    ctx->last_nei_total = nei_total;
    ctx->last_sidx = sidx;
    ctx->last_cell_start = L.cell_start;
    ctx->last_ck = L.ck;
    ctx->last_ck_stride = n;
    ctx->last_nei_off = L.nei_off;
    ctx->last_nei = nei;
    ctx->last_core = L.core;
    ctx->last_cell_label = L.cell_label;
    ctx->last_g = g;
    ctx->last_co = co;
    ctx->last_max_core = max_core;
    ctx->last_key_bits = key_bits;
    ctx->last_walk = walk;
    ctx->last_wide = wide;

    gd_stats& s = ctx->last;
    s.grids = ncell;
    s.neighbor_entries = (int64_t)nei_total;
    s.core_points = ncore;
    s.core_grids = ncc;
    s.dense_grids = H->counts[3];
    s.max_grid_points = 0;
    if (ctx->stats) {
        const StatBlock* sb = ctx->stats_host;
        for (int k = 0; k < kStatSlots; ++k) {
            const MergeStats& m = sb->merge[k];
            s.merge_pairs += (int64_t)m.pairs;
            s.merge_skipped += (int64_t)m.skipped;
            s.merge_tests += (int64_t)m.tests;
            s.merge_yes += (int64_t)m.yes;
            s.merge_iterations += (int64_t)m.iters;
            s.merge_max_iterations = std::max<int64_t>(s.merge_max_iterations, (int64_t)m.max_iters);
            s.merge_distances += (int64_t)m.dists;
            s.merge_set_points += (int64_t)m.set_points;
            s.core_distances += (int64_t)sb->core[k].dists;
            s.core_candidates += (int64_t)sb->core[k].points;
            s.core_neighbor_grids += (int64_t)sb->core[k].grids;
        }
    }
    return GD_OK;
}

int check_params(gd_ctx* ctx, int k, int64_t n, int32_t d, double eps, int32_t minpts, const void* points,
                 const void* labels, const void* core) {
    if (n < 0 || n >= ((int64_t)1 << 31))
        return ctx->fail(GD_EINVAL, "instance %d: n = %lld out of range [0, 2^31)", k, (long long)n);
    if (d < 1 || d > GD_D_MAX) return ctx->fail(GD_EINVAL, "instance %d: d = %d out of range [1, %d]", k, d, GD_D_MAX);
    if (!(eps > 0) || !std::isfinite(eps) || eps != std::floor(eps))
        return ctx->fail(GD_EINVAL, "instance %d: eps = %g must be a positive integer", k, eps);
    if (minpts < 1) return ctx->fail(GD_EINVAL, "instance %d: minpts = %d must be >= 1", k, minpts);
    if (n > 0 && (!points || !labels || !core)) return ctx->fail(GD_EINVAL, "instance %d: NULL device pointer", k);
    return GD_OK;
}

void drop_graph(gd_ctx* ctx) {
    if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
    ctx->gexec = nullptr;
    ctx->gsig.clear();
}

int ensure_inst_capacity(gd_ctx* ctx, int count) {
    if (count <= ctx->inst_cap) return GD_OK;
    // a captured graph reads the instance table through the old pointers
    // (its copy node from the pinned host table, every kernel from the
    // device table): it must never run again
    drop_graph(ctx);
    ++ctx->generation;
    if (ctx->inst_dev) (void)hipFree(ctx->inst_dev);
    if (ctx->inst_host) (void)hipHostFree(ctx->inst_host);
    ctx->inst_dev = nullptr;
    ctx->inst_host = nullptr;
    ctx->inst_cap = 0;
    const int cap = std::max(count, 16);
    if (hipMalloc(&ctx->inst_dev, sizeof(Inst) * cap) != hipSuccess ||
        hipHostMalloc(&ctx->inst_host, sizeof(Inst) * cap, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return ctx->fail(GD_ENOMEM, "instance table allocation failed");
    }
    ctx->inst_cap = cap;
    return GD_OK;
}

// Fill an instance record from the caller's description.
void set_inst(Inst& I, const float* x, int64_t n, int32_t d, double eps, int32_t minpts, int32_t* labels,
              uint8_t* core, int64_t delta) {
    std::memset(&I, 0, sizeof(I));
    I.x = x;
    I.labels = labels;
    I.core = core;
    I.n = n;
    I.d = d;
    // any two valid points are less than 2^25 sqrt(8) < 2^27 apart, so a
    // larger eps clusters exactly as 2^27 does
    I.eps = (int64_t)std::min(eps, (double)kEpsClamp);
    I.T64 = (uint64_t)(I.eps * I.eps);
    I.Tm64 = (uint64_t)((I.eps + delta) * (I.eps + delta));
    // the 32-bit path (eps <= GD_EPS_MAX, eps + delta <= 65535)
    I.T = I.eps <= GD_EPS_MAX ? (uint32_t)I.T64 : 0u;
    I.Tm = I.eps <= GD_EPS_MAX ? (uint32_t)I.Tm64 : 0u;
    I.minpts = minpts;
    for (int j = 0; j < kMaxD; ++j) {
        I.mn[j] = INT_MAX;
        I.mx[j] = INT_MIN;
    }
}

// Global offsets and point tiles of the instances.
void finish_table(gd_ctx* ctx, int count, int* D, int64_t* n, uint32_t* tiles) {
    int64_t off = 0;
    uint32_t t = 0;
    int dm = 1;
    for (int k = 0; k < count; ++k) {
        Inst& I = ctx->inst_host[k];
        I.off = off;
        I.tile0 = t;
        off += I.n;
        t += (uint32_t)((I.n + ctx->tile_pts - 1) / ctx->tile_pts);
        dm = std::max(dm, I.d);
    }
    *D = dm;
    *n = off;
    *tiles = t;
}

// Shape of the batch a graph is valid for: instance sizes and dimensions
// plus the options and host-side choices that change the launch sequence.
// Coordinates, eps, MinPts and the caller's pointers live in the device
// instance table, which the graph re-reads from pinned host memory on every
// replay; the one kernel variant chosen from eps (packed 16-bit coordinate
// differences in core marking, exact only up to kPackedEpsMax) is part of
// the shape, and that kernel also refuses a larger eps on the device.
std::vector<int64_t> batch_signature(const gd_ctx* ctx, int count) {
    std::vector<int64_t> sig;
    sig.reserve(2 * (size_t)count + 7);
    sig.push_back(count);
    int64_t max_eps = 0;
    for (int k = 0; k < count; ++k) max_eps = std::max<int64_t>(max_eps, ctx->inst_host[k].eps);
    sig.push_back(max_eps > GD_EPS_MAX ? 2 : core_mark_packed(max_eps) ? 1 : 0);  // distance width
    sig.push_back(ctx->ldf ? 1 : 0);
    sig.push_back(ctx->proposal_on ? 1 : 0);
    sig.push_back(ctx->tile_pts);
    sig.push_back(ctx->merge_waves);
    sig.push_back(ctx->grid_lanes);
    sig.push_back(ctx->pack_rows ? (ctx->fuse_rows ? 1 : 2) : 0);
    for (int k = 0; k < count; ++k) {
        sig.push_back(ctx->inst_host[k].n);
        sig.push_back(ctx->inst_host[k].d);
    }
    return sig;
}

// Capture a planned run sized from the eager call that just finished.
// Failure to capture is not an error: the call's result is already there.
void capture_graph(gd_ctx* ctx, int count, int D, int64_t n, uint32_t tiles, std::vector<int64_t>&& sig) {
    drop_graph(ctx);
    if (ctx->last_max_core > kMaxCoreBits) return;  // oversized core sets run eagerly
    const gd_stats& e = ctx->last;
    Plan p{};
    const int kb = std::max(ctx->last_key_bits, 1);
    p.key_bits = std::min((kb + 7) / 8 * 8, kb <= 32 ? 32 : kb <= 64 ? 64 : kMaxKeyBits);
    // two-word keys with packed rows keep them in the replay: the headroom
    // stops where the low coordinate bits would no longer fit the word
    if (kb > 32 && kb <= 64 && ctx->pack_rows) {
        const int pb = pack64_width(ctx, count);
        if (pb > 0 && kb + D * pb <= 64) p.key_bits = std::min(p.key_bits, 64 - D * pb);
    }
    p.ncell = std::min<int64_t>(n, e.grids + e.grids / 16 + 1024);
    p.nei = (uint64_t)e.neighbor_entries + (uint64_t)e.neighbor_entries / 16 + 4096;
    p.ncc = std::min<int64_t>(p.ncell, e.core_grids + e.core_grids / 16 + 256);
    p.max_core = std::min<int64_t>(std::min<int64_t>(n, kMaxCoreBits), ctx->last_max_core + ctx->last_max_core / 16 + 64);
    p.walk = ctx->last_walk;
    if (!ctx->gstream) {
        if (hipStreamCreateWithFlags(&ctx->gstream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ctx->gev, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
    }
    const std::string saved_err = ctx->err;
    const uint64_t gen0 = ctx->generation;
    struct Invalidate {  // debug views of the eager call may point into reallocated buffers
        gd_ctx* c;
        uint64_t g;
        ~Invalidate() {
            if (c->generation != g) c->have_last = false;
        }
    } inval{ctx, gen0};
    if (grow(ctx, ctx->cur->nei, (size_t)std::max<uint64_t>(p.nei, 1) * sizeof(uint32_t), ctx->cur->arena.cap) ||
        (p.key_bits <= 64 && grow(ctx, ctx->cur->table, output_table_bytes(table_bits(p.ncell), key_bytes_of(p.key_bits)),
                                  ctx->cur->arena.cap + ctx->cur->nei.cap)) ||
        (ctx->proposal_on && grow(ctx, ctx->cur->sumbuf, sizeof(CellSummary) * (size_t)std::max<int64_t>(p.ncell, 1),
                                  ctx->cur->arena.cap + ctx->cur->nei.cap + ctx->cur->table.cap))) {
        ctx->err = saved_err;
        return;
    }
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(ctx->gstream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    // the captured run only records work: the eager call's counters and
    // debug views stay those of the call that just ran
    const gd_stats saved_last = ctx->last;
    const bool saved_have = ctx->have_last;
    const int rc = run_batch(ctx, count, D, n, tiles, ctx->gstream, &p);
    ctx->last = saved_last;
    ctx->have_last = saved_have;
    const hipError_t ce = hipStreamEndCapture(ctx->gstream, &graph);
    hipGraphExec_t exec = nullptr;
    if (rc == GD_OK && ce == hipSuccess && graph &&
        hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess) {
        ctx->gexec = exec;
        ctx->gsig = std::move(sig);
        ctx->ggen = ctx->generation;
    }
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    ctx->err = saved_err;
}

// One call: replay the captured graph when the batch has its shape, else run
// eagerly (and capture for the next call).  A replay whose data outgrew the
// plan, or that met bad input, is discarded and the call runs eagerly.
int run_call(gd_ctx* ctx, int count, int D, int64_t n, uint32_t tiles, hipStream_t st, bool batched) {
    const bool want = n > 0 && !ctx->stats && !ctx->timing && !ctx->bfs &&
                      (ctx->graph_mode == 2 || (ctx->graph_mode == 1 && batched));
    if (!want) return run_batch(ctx, count, D, n, tiles, st, nullptr);
    std::vector<int64_t> sig = batch_signature(ctx, count);
    if (ctx->gexec && ctx->ggen == ctx->generation && sig == ctx->gsig) {
        GD_TRY(hipEventRecord(ctx->gev, st));
        GD_TRY(hipStreamWaitEvent(ctx->gstream, ctx->gev, 0));
        GD_TRY(hipGraphLaunch(ctx->gexec, ctx->gstream));
        GD_TRY(hipStreamSynchronize(ctx->gstream));
        const Header* H = ctx->hdr_host;
        if (!(H->err & (kErrPlan | kErrNotInteger | kErrKeyBits | kErrNeiOverflow | kErrCoreCap | kErrMergeRunaway))) {
            ctx->have_last = false;  // the debug views describe eager calls only
            std::memset(&ctx->last, 0, sizeof(ctx->last));
            ctx->last.n = n;
            ctx->last.d = D;
            ctx->last.key_bits = ctx->last_key_bits;
            ctx->last.grids = H->ncell;
            ctx->last.neighbor_entries = (int64_t)H->nei_total;
            ctx->last.core_points = H->counts[0];
            ctx->last.core_grids = H->counts[1];
            ctx->last.dense_grids = H->counts[3];
            ctx->last.graph_replays = 1;
            ctx->last.neighbor_walk = ctx->last_walk ? 1 : 0;
            return GD_OK;
        }
        drop_graph(ctx);  // run eagerly below; the next call captures anew
    }
    const int rc = run_batch(ctx, count, D, n, tiles, st, nullptr);
    if (rc == GD_OK) capture_graph(ctx, count, D, n, tiles, std::move(sig));
    return rc;
}

}  // namespace

// ---- Tuning file: a flat JSON object {"<shape key>": {"tile_points": t,
// "merge_waves": w, "grid_lanes": l, "ms": m}, ...} written and read here.

static int ilog2_ceil(int64_t v) {
    int b = 0;
    while (((int64_t)1 << b) < v) ++b;
    return b;
}

// Shape key of a batch: instance count, total points and largest n as powers
// of two (rounded up), and the range of d.
static std::string tuning_key(const gd_instance* inst, int count) {
    int64_t total = 0, nmax = 0;
    int dmin = GD_D_MAX, dmax = 1;
    for (int k = 0; k < count; ++k) {
        total += inst[k].n;
        nmax = std::max<int64_t>(nmax, inst[k].n);
        dmin = std::min(dmin, (int)inst[k].d);
        dmax = std::max(dmax, (int)inst[k].d);
    }
    char buf[128];
    std::snprintf(buf, sizeof(buf), "count=%d;points=2^%d;nmax=2^%d;d=%d-%d", count, ilog2_ceil(total),
                  ilog2_ceil(nmax), dmin, dmax);
    return buf;
}

// Entries of a tuning file (an unreadable file or entry is skipped).
static std::map<std::string, gd_tuning> read_tuning_file(const std::string& path) {
    std::map<std::string, gd_tuning> out;
    FILE* f = std::fopen(path.c_str(), "rb");
    if (!f) return out;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    std::fclose(f);
    auto field = [](const std::string& obj, const char* name, double& v) -> bool {
        const std::string tag = std::string("\"") + name + "\"";
        const size_t p = obj.find(tag);
        if (p == std::string::npos) return false;
        const size_t c = obj.find(':', p + tag.size());
        if (c == std::string::npos) return false;
        char* end = nullptr;
        v = std::strtod(obj.c_str() + c + 1, &end);
        return end != obj.c_str() + c + 1;
    };
    size_t pos = text.find('{');
    while (pos != std::string::npos) {
        const size_t k0 = text.find('"', pos + 1);
        if (k0 == std::string::npos) break;
        const size_t k1 = text.find('"', k0 + 1);
        const size_t o0 = k1 == std::string::npos ? k1 : text.find('{', k1);
        const size_t o1 = o0 == std::string::npos ? o0 : text.find('}', o0);
        if (o1 == std::string::npos) break;
        const std::string key = text.substr(k0 + 1, k1 - k0 - 1), obj = text.substr(o0, o1 - o0 + 1);
        double t = 0, w = 0, l = 0, ms = 0;
        if (field(obj, "tile_points", t) && field(obj, "merge_waves", w) && field(obj, "grid_lanes", l)) {
            (void)field(obj, "ms", ms);
            out[key] = gd_tuning{(int32_t)t, (int32_t)w, (int32_t)l, ms};
        }
        pos = o1;
    }
    return out;
}

static bool write_tuning_file(const std::string& path, const std::map<std::string, gd_tuning>& entries) {
    const std::string tmp = path + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& e : entries) {
        std::fprintf(f, "  \"%s\": {\"tile_points\": %d, \"merge_waves\": %d, \"grid_lanes\": %d, \"ms\": %.4f}%s\n",
                     e.first.c_str(), e.second.tile_points, e.second.merge_waves, e.second.grid_lanes, e.second.ms,
                     ++i < entries.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path.c_str()) == 0;
}

static bool valid_tuning(const gd_tuning& t) {
    return t.tile_points >= 256 && t.tile_points <= 65536 && t.tile_points % 256 == 0 &&
           (t.merge_waves == 1 || t.merge_waves == 2 || t.merge_waves == 4) &&
           (t.grid_lanes == 0 || t.grid_lanes == 16 || t.grid_lanes == 64);
}

extern "C" {

int gd_create(gd_ctx** out, int device) {
    if (!out) return GD_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return GD_EINVAL;
    gd_ctx* ctx = new gd_ctx();
    ctx->device = device;
    bool ok;
    {
        DeviceGuard guard(device);
        ok = guard.ok && hipMalloc(&ctx->hdr_dev, sizeof(Header)) == hipSuccess &&
             hipHostMalloc(&ctx->hdr_host, sizeof(Header), hipHostMallocDefault) == hipSuccess &&
             hipMalloc(&ctx->stats_dev, sizeof(StatBlock)) == hipSuccess &&
             hipHostMalloc(&ctx->stats_host, sizeof(StatBlock), hipHostMallocDefault) == hipSuccess &&
             hipMalloc(&ctx->proposal_dev, sizeof(__half) * kParams) == hipSuccess &&
             hipMalloc(&ctx->counter_dev, sizeof(unsigned long long)) == hipSuccess &&
             ensure_inst_capacity(ctx, 16) == GD_OK;
        // with the device current: this device's copy of the scratch array
        if (ok) ctx->scratch = scratch_address(device);
        if (ok) {
            ctx->events_ok = true;
            for (int p = 0; p < P_COUNT; ++p)
                for (int k = 0; k < 2; ++k)
                    if (hipEventCreate(&ctx->ev[p][k]) != hipSuccess) ctx->events_ok = false;
        }
    }
    if (!ok) {
        gd_destroy(ctx);
        return GD_EDEVICE;
    }
    *out = ctx;
    return GD_OK;
}

void gd_destroy(gd_ctx* ctx) {
    if (!ctx) return;
    DeviceGuard guard(ctx->device);
    if (ctx->own.arena.p) (void)hipFree(ctx->own.arena.p);
    if (ctx->own.nei.p) (void)hipFree(ctx->own.nei.p);
    if (ctx->hdr_dev) (void)hipFree(ctx->hdr_dev);
    if (ctx->hdr_host) (void)hipHostFree(ctx->hdr_host);
    if (ctx->stats_dev) (void)hipFree(ctx->stats_dev);
    if (ctx->stats_host) (void)hipHostFree(ctx->stats_host);
    if (ctx->inst_dev) (void)hipFree(ctx->inst_dev);
    if (ctx->inst_host) (void)hipHostFree(ctx->inst_host);
    if (ctx->proposal_dev) (void)hipFree(ctx->proposal_dev);
    if (ctx->counter_dev) (void)hipFree(ctx->counter_dev);
    if (ctx->own.sumbuf.p) (void)hipFree(ctx->own.sumbuf.p);
    if (ctx->own.table.p) (void)hipFree(ctx->own.table.p);
    if (ctx->own.huge.p) (void)hipFree(ctx->own.huge.p);
    drop_graph(ctx);
    if (ctx->gev) (void)hipEventDestroy(ctx->gev);
    if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
    for (int p = 0; p < P_COUNT; ++p)
        for (int k = 0; k < 2; ++k)
            if (ctx->ev[p][k]) (void)hipEventDestroy(ctx->ev[p][k]);
    delete ctx;
}

int dbscan(gd_ctx* ctx, const float* points, int64_t n, int32_t d, double eps, int32_t minpts, int32_t* labels,
           uint8_t* core_flags, void* stream) {
    if (!ctx) return GD_EINVAL;
    ctx->err.clear();
    int rc = check_params(ctx, 0, n, d, eps, minpts, points, labels, core_flags);
    if (rc) return rc;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return ctx->fail(GD_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    set_inst(ctx->inst_host[0], points, n, d, eps, minpts, labels, core_flags, ctx->approx_delta);
    int D;
    int64_t total;
    uint32_t tiles;
    finish_table(ctx, 1, &D, &total, &tiles);
    return run_call(ctx, 1, D, total, tiles, (hipStream_t)stream, false);
}

int dbscan_noalloc(gd_ctx* ctx, const float* points, int64_t n, int32_t d, double eps, int32_t minpts,
                   int32_t* labels, uint8_t* core_flags, void* stream) {
    if (!ctx) return GD_EINVAL;
    ctx->err.clear();
    int rc = check_params(ctx, 0, n, d, eps, minpts, points, labels, core_flags);
    if (rc) return rc;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return ctx->fail(GD_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    if (!ctx->scratch) return ctx->fail(GD_EDEVICE, "dbscan_noalloc: the scratch array's device address is unknown");
    set_inst(ctx->inst_host[0], points, n, d, eps, minpts, labels, core_flags, ctx->approx_delta);
    int D;
    int64_t total;
    uint32_t tiles;
    finish_table(ctx, 1, &D, &total, &tiles);
    const size_t need = carve(nullptr, total, D, tiles).bytes;
    if (need > (size_t)GD_NOALLOC_SCRATCH_BYTES)
        return ctx->fail(GD_ENOMEM,
                         "dbscan_noalloc: n = %lld at d = %d needs %zu bytes of workspace before its neighbour "
                         "lists; the fixed scratch holds %llu",
                         (long long)n, d, need, (unsigned long long)GD_NOALLOC_SCRATCH_BYTES);
    // every buffer of this call comes from the scratch array, in order;
    // nothing is allocated and no graph is captured or replayed
    Bufs view{};
    ctx->cur = &view;
    ctx->bump_base = ctx->scratch;
    ctx->bump_cap = (size_t)GD_NOALLOC_SCRATCH_BYTES;
    ctx->bump_used = 0;
    rc = run_batch(ctx, 1, D, total, tiles, (hipStream_t)stream, nullptr);
    ctx->cur = &ctx->own;
    ctx->bump_base = nullptr;
    return rc;
}

int dbscan_batched(gd_ctx* ctx, const gd_instance* inst, int32_t count, void* stream) {
    if (!ctx) return GD_EINVAL;
    ctx->err.clear();
    if (count < 0 || (count > 0 && !inst)) return ctx->fail(GD_EINVAL, "bad instance array");
    if (count > GD_BATCH_MAX) return ctx->fail(GD_EINVAL, "count = %d exceeds %d", count, GD_BATCH_MAX);
    int64_t total = 0;
    for (int k = 0; k < count; ++k) {
        const gd_instance& q = inst[k];
        int rc = check_params(ctx, k, q.n, q.d, q.eps, q.minpts, q.points, q.labels, q.core_flags);
        if (rc) return rc;
        total += q.n;
    }
    if (total >= ((int64_t)1 << 31)) return ctx->fail(GD_EINVAL, "batch holds %lld points (>= 2^31)", (long long)total);
    if (count == 0) return GD_OK;
    DeviceGuard guard(ctx->device);
    if (!guard.ok) return ctx->fail(GD_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    int rc = ensure_inst_capacity(ctx, count);
    if (rc) return rc;
    for (int k = 0; k < count; ++k) {
        const gd_instance& q = inst[k];
        set_inst(ctx->inst_host[k], q.points, q.n, q.d, q.eps, q.minpts, q.labels, q.core_flags, ctx->approx_delta);
    }
    int D;
    uint32_t tiles;
    finish_table(ctx, count, &D, &total, &tiles);
    return run_call(ctx, count, D, total, tiles, (hipStream_t)stream, true);
}

int gd_set_tuning_file(gd_ctx* ctx, const char* path) {
    if (!ctx) return GD_EINVAL;
    ctx->err.clear();
    ctx->tuning_file = path ? path : "";
    return GD_OK;
}

int gd_autotune(gd_ctx* ctx, const gd_instance* inst, int32_t count, void* stream, gd_tuning* results,
                int32_t max_results, int32_t* n_results) {
    if (!ctx) return GD_EINVAL;
    ctx->err.clear();
    if (n_results) *n_results = 0;
    if (count < 0 || (count > 0 && !inst)) return ctx->fail(GD_EINVAL, "bad batch descriptor");
    const std::string key = tuning_key(inst, count);
    std::map<std::string, gd_tuning> file;
    if (!ctx->tuning_file.empty()) {
        file = read_tuning_file(ctx->tuning_file);
        const auto it = file.find(key);
        if (it != file.end() && valid_tuning(it->second)) {
            ctx->tile_pts = it->second.tile_points;
            ctx->merge_waves = it->second.merge_waves;
            ctx->grid_lanes = it->second.grid_lanes;
            return GD_OK;
        }
    }
    static const int kTiles[] = {1024, 4096};
    static const int kWaves[] = {1, 2, 4};
    static const int kLanes[] = {16, 64};
    const int saved_tile = ctx->tile_pts, saved_waves = ctx->merge_waves, saved_lanes = ctx->grid_lanes;
    const int saved_graph = ctx->graph_mode;
    const bool saved_stats = ctx->stats, saved_timing = ctx->timing;
    ctx->graph_mode = 0;
    ctx->stats = false;
    ctx->timing = false;
    gd_tuning best{saved_tile, saved_waves, saved_lanes, 1e300};
    int k = 0, rc = GD_OK;
    for (int tile : kTiles) {
        for (int waves : kWaves) {
            for (int lanes : kLanes) {
                ctx->tile_pts = tile;
                ctx->merge_waves = waves;
                ctx->grid_lanes = lanes;
                double t[4];
                for (int rep = 0; rep < 4 && rc == GD_OK; ++rep) {  // the first call also warms the workspace
                    const auto t0 = std::chrono::steady_clock::now();
                    rc = dbscan_batched(ctx, inst, count, stream);
                    const auto t1 = std::chrono::steady_clock::now();
                    t[rep] = std::chrono::duration<double, std::milli>(t1 - t0).count();
                }
                if (rc != GD_OK) break;
                std::sort(t + 1, t + 4);
                const gd_tuning row{tile, waves, lanes, t[2]};
                if (results && k < max_results) results[k] = row;
                ++k;
                if (row.ms < best.ms) best = row;
            }
            if (rc != GD_OK) break;
        }
        if (rc != GD_OK) break;
    }
    ctx->graph_mode = saved_graph;
    ctx->stats = saved_stats;
    ctx->timing = saved_timing;
    if (n_results) *n_results = std::min(k, max_results);
    if (rc != GD_OK) {
        ctx->tile_pts = saved_tile;
        ctx->merge_waves = saved_waves;
        ctx->grid_lanes = saved_lanes;
        return rc;
    }
    ctx->tile_pts = best.tile_points;
    ctx->merge_waves = best.merge_waves;
    ctx->grid_lanes = best.grid_lanes;
    if (!ctx->tuning_file.empty()) {
        file[key] = best;
        if (!write_tuning_file(ctx->tuning_file, file))
            return ctx->fail(GD_EINVAL, "cannot write the tuning file %s", ctx->tuning_file.c_str());
    }
    return GD_OK;
}

int gd_set_option(gd_ctx* ctx, int option, int64_t value) {
    if (!ctx) return GD_EINVAL;
    switch (option) {
        case GD_OPT_STATS: ctx->stats = value != 0; return GD_OK;
        case GD_OPT_LDF_ORDER:
            ctx->ldf = value != 0;
            ctx->bfs = false;
            return GD_OK;
        case GD_OPT_MERGE_ORDER:
            if (value < 0 || value > 2) return ctx->fail(GD_EINVAL, "merge order must be 0, 1 or 2");
            ctx->ldf = value == 1;
            ctx->bfs = value == 2;
            return GD_OK;
        case GD_OPT_TIMING: ctx->timing = value != 0; return GD_OK;
        case GD_OPT_TILE_POINTS:
            if (value < 256 || value > 65536 || value % 256)
                return ctx->fail(GD_EINVAL, "tile size must be a multiple of 256 in [256, 65536]");
            ctx->tile_pts = (int)value;
            return GD_OK;
        case GD_OPT_MERGE_WAVES:
            if (value != 1 && value != 2 && value != 4) return ctx->fail(GD_EINVAL, "merge waves must be 1, 2 or 4");
            ctx->merge_waves = (int)value;
            return GD_OK;
        case GD_OPT_GRID_LANES:
            if (value != 0 && value != 16 && value != 64)
                return ctx->fail(GD_EINVAL, "lanes per grid must be 0, 16 or 64");
            ctx->grid_lanes = (int)value;
            return GD_OK;
        case GD_OPT_PACKED_ROWS:
            if (value < 0 || value > 2) return ctx->fail(GD_EINVAL, "packed rows must be 0, 1 or 2");
            ctx->pack_rows = value != 0;
            ctx->fuse_rows = value == 1;
            return GD_OK;
        case GD_OPT_GRAPH:
            if (value < 0 || value > 2) return ctx->fail(GD_EINVAL, "graph mode must be 0, 1 or 2");
            ctx->graph_mode = (int)value;
            if (value == 0) {
                DeviceGuard guard(ctx->device);
                drop_graph(ctx);
            }
            return GD_OK;
        case GD_OPT_NEIGHBOR_QUERY:
            if (value < 0 || value > 3) return ctx->fail(GD_EINVAL, "neighbour query must be 0, 1, 2 or 3");
            ctx->nei_query = value == 0 ? kNeiAuto : value == 3 ? (int)kNeiTree : (int)value;
            return GD_OK;
        case GD_OPT_APPROX_DELTA:
            if (value < 0 || value > kApproxDeltaMax)
                return ctx->fail(GD_EINVAL, "approximation delta must be in [0, %d]", kApproxDeltaMax);
            ctx->approx_delta = value;
            return GD_OK;
        case GD_OPT_NEIGHBOR_MODE:
            if (value < 0 || value > 2) return ctx->fail(GD_EINVAL, "neighbour mode must be 0, 1 or 2");
            ctx->nei_mode = (int)value;
            return GD_OK;
        case GD_OPT_WORKSPACE_LIMIT:
            if (value < 0) return ctx->fail(GD_EINVAL, "workspace limit must be >= 0");
            ctx->ws_limit = value;
            return GD_OK;
        default: return ctx->fail(GD_EINVAL, "unknown option %d", option);
    }
}

int gd_get_stats(gd_ctx* ctx, gd_stats* out) {
    if (!ctx || !out) return GD_EINVAL;
    *out = ctx->last;
    return GD_OK;
}

static int copy_d2h(gd_ctx* ctx, void* dst, const void* src, size_t bytes) {
    if (!dst || bytes == 0) return GD_OK;
    if (hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost) != hipSuccess)
        return ctx->fail(GD_EDEVICE, "device-to-host copy failed");
    return GD_OK;
}

int gd_debug_grids(gd_ctx* ctx, int64_t* n_grids, uint32_t* sorted_index, uint32_t* grid_start, int32_t* grid_ids) {
    if (!ctx) return GD_EINVAL;
    if (!ctx->have_last) return ctx->fail(GD_EINVAL, "no successful dbscan() call to inspect");
    DeviceGuard guard(ctx->device);
    if (n_grids) *n_grids = ctx->last_ncell;
    const int64_t n = ctx->last_n, nc = ctx->last_ncell;
    int rc;
    if ((rc = copy_d2h(ctx, sorted_index, ctx->last_sidx, sizeof(uint32_t) * n))) return rc;
    if ((rc = copy_d2h(ctx, grid_start, ctx->last_cell_start, sizeof(uint32_t) * (nc + 1)))) return rc;
    if (grid_ids) {
        // rows 1..D of the identifier table (row 0 is the instance)
        std::vector<int32_t> col(nc);
        for (int j = 0; j < ctx->last_d; ++j) {
            if ((rc = copy_d2h(ctx, col.data(), ctx->last_ck + (int64_t)(j + 1) * ctx->last_ck_stride,
                               sizeof(int32_t) * nc)))
                return rc;
            for (int64_t c = 0; c < nc; ++c) grid_ids[c * ctx->last_d + j] = col[c];
        }
    }
    return GD_OK;
}

int gd_debug_neighbors(gd_ctx* ctx, uint64_t* offsets, uint32_t* neighbors) {
    if (!ctx) return GD_EINVAL;
    if (!ctx->have_last) return ctx->fail(GD_EINVAL, "no successful dbscan() call to inspect");
    if (ctx->last_walk)
        return ctx->fail(GD_EUNSUPPORTED, "the last call walked the grid tree instead of writing every list "
                                          "(GD_OPT_NEIGHBOR_MODE = 1 keeps them)");
    DeviceGuard guard(ctx->device);
    int rc;
    if ((rc = copy_d2h(ctx, offsets, ctx->last_nei_off, sizeof(uint64_t) * (ctx->last_ncell + 1)))) return rc;
    return copy_d2h(ctx, neighbors, ctx->last_nei, sizeof(uint32_t) * ctx->last_nei_total);
}

int gd_debug_core(gd_ctx* ctx, uint8_t* core_flags_sorted, int32_t* grid_label) {
    if (!ctx) return GD_EINVAL;
    if (!ctx->have_last) return ctx->fail(GD_EINVAL, "no successful dbscan() call to inspect");
    DeviceGuard guard(ctx->device);
    int rc;
    if ((rc = copy_d2h(ctx, core_flags_sorted, ctx->last_core, ctx->last_n))) return rc;
    return copy_d2h(ctx, grid_label, ctx->last_cell_label, sizeof(int32_t) * ctx->last_ncell);
}

int gd_merge_test(gd_ctx* ctx, const int32_t* points, int64_t m, int32_t d, double eps, const uint32_t* pairs,
                  int64_t npairs, uint8_t* answers, uint32_t* iterations, void* stream) {
    if (!ctx) return GD_EINVAL;
    ctx->err.clear();
    if (d < 1 || d > GD_D_MAX) return ctx->fail(GD_EINVAL, "d = %d out of range [1, %d]", d, GD_D_MAX);
    if (!(eps > 0) || !std::isfinite(eps) || eps != std::floor(eps))
        return ctx->fail(GD_EINVAL, "eps = %g must be a positive integer", eps);
    if (eps > (double)kEpsClamp) return ctx->fail(GD_ERANGE, "eps = %g exceeds 2^27", eps);
    if (m < 0 || npairs < 0) return ctx->fail(GD_EINVAL, "negative size");
    if (npairs == 0) return GD_OK;
    if (!points || !pairs || !answers) return ctx->fail(GD_EINVAL, "NULL device pointer");
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    std::vector<uint32_t> hp((size_t)npairs * 4);
    GD_TRY(hipMemcpyAsync(hp.data(), pairs, hp.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    GD_TRY(hipStreamSynchronize(st));
    uint32_t mx = 1;
    for (int64_t r = 0; r < npairs; ++r) {
        for (int s = 0; s < 2; ++s) {
            const uint64_t b = hp[4 * r + 2 * s], c = hp[4 * r + 2 * s + 1];
            if (c < 1 || c > (uint64_t)kMaxCoreBits || b + c > (uint64_t)m)
                return ctx->fail(GD_EINVAL, "pair %lld: run [%llu, +%llu) invalid for m = %lld", (long long)r,
                                 (unsigned long long)b, (unsigned long long)c, (long long)m);
            mx = std::max<uint32_t>(mx, (uint32_t)c);
        }
    }
    int32_t* rows = nullptr;
    if (hipMalloc(&rows, sizeof(int32_t) * (size_t)row_stride(d) * (size_t)std::max<int64_t>(m, 1)) != hipSuccess) {
        (void)hipGetLastError();
        return ctx->fail(GD_ENOMEM, "row buffer allocation failed");
    }
    hipError_t e = launch_merge_pairs(points, m, d, rows, pairs, npairs, (int64_t)eps, mx, answers, iterations, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(rows);
    if (e != hipSuccess) return ctx->fail(GD_EDEVICE, "merge test failed: %s", hipGetErrorString(e));
    return GD_OK;
}

int gd_set_proposal(gd_ctx* ctx, const uint16_t* fp16_params) {
    if (!ctx) return GD_EINVAL;
    ctx->err.clear();
    if (!fp16_params) {
        ctx->proposal_on = false;
        return GD_OK;
    }
    DeviceGuard guard(ctx->device);
    if (hipMemcpy(ctx->proposal_dev, fp16_params, sizeof(__half) * kParams, hipMemcpyHostToDevice) != hipSuccess)
        return ctx->fail(GD_EDEVICE, "copy of the proposal weights failed");
    ctx->proposal_on = true;
    return GD_OK;
}

int gd_proposal_harvest(gd_ctx* ctx, uint32_t seed, uint32_t keep_mod, int64_t cap, uint16_t* features,
                        float* targets, float* costs, int64_t* count, void* stream) {
    if (!ctx) return GD_EINVAL;
    ctx->err.clear();
    if (!ctx->have_last) return ctx->fail(GD_EINVAL, "no successful dbscan() call to harvest from");
    if (ctx->last_walk)
        return ctx->fail(GD_EUNSUPPORTED, "harvesting needs the neighbour lists of every grid "
                                          "(GD_OPT_NEIGHBOR_MODE = 1)");
    if (ctx->last_wide)
        return ctx->fail(GD_EUNSUPPORTED, "harvesting takes eps <= %d (the scorer's 32-bit path)", GD_EPS_MAX);
    if (keep_mod < 1 || cap < 0 || (cap > 0 && (!features || !targets)) || !count)
        return ctx->fail(GD_EINVAL, "bad harvest arguments");
    DeviceGuard guard(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const GridView& g = ctx->last_g;
    int rc;
    if ((rc = grow(ctx, ctx->cur->sumbuf, sizeof(CellSummary) * (size_t)std::max<int64_t>(g.ncell, 1),
                   ctx->cur->arena.cap + ctx->cur->nei.cap)))
        return rc;
    CellSummary* sum = (CellSummary*)ctx->cur->sumbuf.p;
    GD_TRY(fill<unsigned long long>(ctx->counter_dev, 1, 0ull, st));
    GD_TRY(launch_summaries(g, ctx->last_co, sum, st));
    GD_TRY(launch_harvest(g, ctx->last_co, sum, ctx->last_nei_off, ctx->last_nei, seed, keep_mod, cap,
                          ctx->last_max_core, (__half*)features, targets, costs, ctx->counter_dev, st));
    unsigned long long got = 0;
    GD_TRY(hipMemcpyAsync(&got, ctx->counter_dev, sizeof(got), hipMemcpyDeviceToHost, st));
    GD_TRY(hipStreamSynchronize(st));
    *count = (int64_t)std::min<unsigned long long>(got, (unsigned long long)cap);
    return GD_OK;
}

int gd_mlp_train(gd_ctx* ctx, const uint16_t* features, const float* targets, int64_t S, const uint32_t* order,
                 int32_t steps, int32_t batch, float lr, int32_t adam_t0, float* params, float* adam_m,
                 float* adam_v, float* loss, uint16_t* blob, void* stream) {
    if (!ctx) return GD_EINVAL;
    ctx->err.clear();
    if (S < 1 || steps < 0 || batch < 1 || !features || !targets || !order || !params || !adam_m || !adam_v ||
        !(lr > 0.f) || adam_t0 < 0)
        return ctx->fail(GD_EINVAL, "bad training arguments");
    DeviceGuard guard(ctx->device);
    TrainArgs a{};
    a.x = (const __half*)features;
    a.t = targets;
    a.order = order;
    a.steps = steps;
    a.batch = batch;
    a.lr = lr;
    a.adam_t0 = adam_t0;
    a.params = params;
    a.m = adam_m;
    a.v = adam_v;
    a.loss = loss;
    a.grad = nullptr;
    a.update = 1;
    a.blob = (__half*)blob;
    GD_TRY(launch_mlp_train(a, (hipStream_t)stream));
    GD_TRY(hipStreamSynchronize((hipStream_t)stream));
    return GD_OK;
}

int gd_mlp_grad(gd_ctx* ctx, const uint16_t* features, const float* targets, const uint32_t* order, int32_t batch,
                const float* params, float* grad, float* loss, void* stream) {
    if (!ctx) return GD_EINVAL;
    ctx->err.clear();
    if (batch < 1 || !features || !targets || !order || !params || !grad)
        return ctx->fail(GD_EINVAL, "bad gradient arguments");
    DeviceGuard guard(ctx->device);
    TrainArgs a{};
    a.x = (const __half*)features;
    a.t = targets;
    a.order = order;
    a.steps = 1;
    a.batch = batch;
    a.lr = 1.f;
    a.params = const_cast<float*>(params);  // not written: update = 0
    a.m = nullptr;
    a.v = nullptr;
    a.loss = loss;
    a.grad = grad;
    a.update = 0;
    a.blob = nullptr;
    GD_TRY(launch_mlp_train(a, (hipStream_t)stream));
    GD_TRY(hipStreamSynchronize((hipStream_t)stream));
    return GD_OK;
}

int gd_mlp_forward(gd_ctx* ctx, const uint16_t* features, int64_t B, const uint16_t* blob, float* logits,
                   void* stream) {
    if (!ctx) return GD_EINVAL;
    ctx->err.clear();
    if (B < 0 || (B > 0 && (!features || !blob || !logits))) return ctx->fail(GD_EINVAL, "bad forward arguments");
    DeviceGuard guard(ctx->device);
    GD_TRY(launch_mlp_forward((const __half*)features, B, (const __half*)blob, logits, (hipStream_t)stream));
    GD_TRY(hipStreamSynchronize((hipStream_t)stream));
    return GD_OK;
}

int gd_get_phase_times(gd_ctx* ctx, double* ms, int32_t count) {
    if (!ctx || (!ms && count > 0) || count < 0) return GD_EINVAL;
    for (int p = 0; p < count; ++p) ms[p] = p < P_COUNT ? ctx->phase_ms[p] : 0.0;
    return GD_OK;
}

const char* gd_phase_name(int32_t i) { return (i >= 0 && i < P_COUNT) ? kPhaseNames[i] : nullptr; }

const char* gd_last_error(gd_ctx* ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

const char* gd_status_string(int status) {
    switch (status) {
        case GD_OK: return "GD_OK";
        case GD_EINVAL: return "GD_EINVAL";
        case GD_ERANGE: return "GD_ERANGE";
        case GD_ENOMEM: return "GD_ENOMEM";
        case GD_EDEVICE: return "GD_EDEVICE";
        case GD_EUNSUPPORTED: return "GD_EUNSUPPORTED";
        default: return "unknown status";
    }
}

}  // extern "C"
