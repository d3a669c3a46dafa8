// The neighbouring-grid query of Algorithm 3 (Section 4.2.2, Eq. (2)) as a
// walk that hands each neighbour to its consumer as soon as it is found,
// instead of writing Nei(g) out first.
//
// A query for grid g descends the grid tree level by level.  At level l it
// keeps the children whose key k satisfies |k - g_l| <= w, with
//   offset += max(|k - g_l| - 1, 0)^2                       (Eq. (2))
// and drops a node once offset >= d; the window shrinks with the budget
// left (w = 1 + isqrt(d - 1 - offset)), which keeps exactly the nodes the
// paper's fixed window +-ceil(sqrt(d)) keeps after pruning.  The first
// child in a window comes from a binary search over the node's contiguous,
// ascending children (the role of the paper's hash table h).
//
// Two forms:
//   full  - every neighbour g' != g.  Level 1 is taken centre-out (key
//           offsets 0, -1, +1, -2, +2, ...), so nearer grids tend to come
//           first, as the paper's offset order intends for early exit;
//   upper - only neighbours whose identifier is lexicographically larger
//           than g's (grid index above g's), so that a pairwise step can
//           take every unordered pair once, from its lower grid.
// The visitor returns false to stop the walk (early exit).
#pragma once

#include "launch.hpp"

namespace gd {

// w = 1 + isqrt(budget - 1) for a budget of 1..9 (budgets never exceed the
// instance dimension, at most 8): isqrt(b - 1) counts k >= 1 with k^2 <= b - 1.
__device__ __forceinline__ int walk_window(int budget) {
    return 1 + (budget >= 2 ? 1 : 0) + (budget >= 5 ? 1 : 0);
}

// First index in [lo, hi) whose key is >= want.
__device__ __forceinline__ uint32_t walk_lower(const int32_t* __restrict__ key, uint32_t lo, uint32_t hi, int32_t want) {
    while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if (key[m] < want) lo = m + 1; else hi = m;
    }
    return lo;
}

// Levels L..D below a node whose children are [lo, hi).  gt: the path so
// far is already above g's identifier (always true in the full form).
template <int D, int L, typename V>
__device__ __forceinline__ bool walk_levels(const TreeView& t, const int32_t (&g)[D + 1], int dk, uint32_t lo,
                                            uint32_t hi, int off, bool gt, V& visit) {
    const int win = walk_window(dk - off);
    const int32_t* __restrict__ key = t.key[L];
    uint32_t a = walk_lower(key, lo, hi, gt ? g[L] - win : g[L]);
    for (; a < hi; ++a) {
        const int32_t dl = key[a] - g[L];
        if (dl > win) break;
        const int gap = (dl < 0 ? -dl : dl) - 1;
        const int o = off + (gap > 0 ? gap * gap : 0);
        if (o >= dk) continue;
        const bool ngt = gt || dl > 0;
        if constexpr (L == D) {
            if (!ngt) continue;  // g itself
            if (!visit(a, o)) return false;
        } else {
            if (!walk_levels<D, L + 1>(t, g, dk, t.child[L][a], t.child[L][a + 1], o, ngt, visit)) return false;
        }
    }
    return true;
}

// Neighbours of the grid with identifiers g[1..D] in instance g[0] (dk: the
// instance's own dimension; rows beyond it are 0).  In the full form the
// visitor sees g itself too and must skip it (the caller knows its index).
template <int D, typename V>
__device__ __forceinline__ void tree_walk(const TreeView& t, const int32_t (&g)[D + 1], int dk, bool upper, V& visit) {
    const uint32_t a0 = walk_lower(t.key[0], 0, t.level_count[0], g[0]);
    const uint32_t lo1 = t.child[0][a0], hi1 = t.child[0][a0 + 1];
    const int32_t* __restrict__ key1 = t.key[1];
    const int w1 = walk_window(dk);
    for (int s = 0; s <= 2 * w1; ++s) {
        const int delta = (s & 1) ? -((s + 1) >> 1) : (s >> 1);  // 0, -1, +1, -2, +2, ...
        if (upper && delta < 0) continue;
        const int32_t want = g[1] + delta;
        const uint32_t a = walk_lower(key1, lo1, hi1, want);
        if (a >= hi1 || key1[a] != want) continue;
        const int gap = (delta < 0 ? -delta : delta) - 1;
        const int o = gap > 0 ? gap * gap : 0;
        if (o >= dk) continue;
        const bool gt = !upper || delta > 0;
        if constexpr (D == 1) {
            if (upper && !gt) continue;
            if (!visit(a, o)) return;
        } else {
            if (!walk_levels<D, 2>(t, g, dk, t.child[1][a], t.child[1][a + 1], o, gt, visit)) return;
        }
    }
}

template <int D>
__device__ __forceinline__ void load_grid_key(const GridView& gv, int64_t c, int32_t (&g)[D + 1]) {
#pragma unroll
    for (int j = 0; j <= D; ++j) g[j] = gv.ck[(int64_t)j * gv.ck_stride + c];
}

}  // namespace gd
