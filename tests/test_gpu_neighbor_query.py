"""Neighbour queries (GD_OPT_NEIGHBOR_QUERY): the grid tree of Algorithm 3
with offset-ordered lists, the grid tree in walk order, direct hashing of
every candidate identifier, and the default that picks between the first
two by the grids' mean size.  Each must produce Nei(g) exactly as defined
(Eq. (2), g excluded), ordered by offset where promised, and the same
clustering as the oracle."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import steps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

AUTO, TREE_WALK_ORDER, HASH, TREE = 0, 1, 2, 3


@pytest.fixture(scope="module")
def G():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G


def ctx_for(G, query):
    c = G.Context(0)
    c.set_option(G.GD_OPT_NEIGHBOR_MODE, 1)  # lists for every grid (the debug view reads them)
    c.set_option(G.GD_OPT_NEIGHBOR_QUERY, query)
    return c


def run(ctx, x, eps, minpts):
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    lab, core = ctx.dbscan(t, eps, minpts)
    return lab.cpu().numpy(), core.cpu().numpy()


@pytest.mark.parametrize("query", [TREE, TREE_WALK_ORDER, HASH, AUTO])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6])
def test_lists_match_definition(G, query, d):
    rng = np.random.default_rng(70 + d)
    n = 1500 if d < 5 else 700
    x = rng.integers(0, 1200, size=(n, d)).astype(np.int32)
    eps = 150
    ctx = ctx_for(G, query)
    print(f"case query={query} d={d}", flush=True)
    run(ctx, x, eps, 3)
    sidx, gs, ids = ctx.debug_grids()
    off, nei = ctx.debug_neighbors()
    want, _ = steps.neighbor_grids(ids)
    for g in range(len(ids)):
        got = nei[off[g]:off[g + 1]].astype(np.int64)
        assert sorted(got.tolist()) == want[g].tolist(), f"grid {g}"
        if query in (TREE, HASH):
            o = [steps.grid_offset(ids[g], ids[h]) for h in got]
            assert o == sorted(o), f"grid {g}: not ordered by offset"
    ctx.close()


@pytest.mark.parametrize("query", [TREE_WALK_ORDER, HASH, AUTO])
@pytest.mark.parametrize("seed", range(6))
def test_random_vs_brute(G, query, seed):
    rng = np.random.default_rng(900 + seed)
    d = 1 + seed % 6
    n = int(rng.integers(1, 800))
    domain = int(rng.integers(20, 400))
    x = rng.integers(0, domain, size=(n, d)).astype(np.int32) - domain // 3
    eps = int(rng.integers(1, max(2, domain // 4)))
    while sum(int(v).bit_length() for v in steps.cell_ids(x, eps).max(axis=0)) > 64:
        eps += 1
    minpts = int(rng.choice([1, 2, 4, 9, n + 1]))
    ctx = ctx_for(G, query)
    print(f"case query={query} seed={seed} n={n} d={d} eps={eps} minpts={minpts}", flush=True)
    lab, core = run(ctx, x, eps, minpts)
    wl, wc = oracle.dbscan_brute(x, eps, minpts)
    assert np.array_equal(core, wc) and np.array_equal(lab, wl)
    ctx.close()


@pytest.mark.parametrize("name,n", [("cfg1", 150_000), ("cfg2", 150_000), ("cfg0", 10_000)])
def test_workloads(G, name, n):
    w = W.WORKLOADS[name].with_n(n)
    x = W.make_points(w)
    want = oracle.dbscan(x, w.eps, w.minpts)
    for query in (TREE_WALK_ORDER, HASH):
        ctx = ctx_for(G, query)
        print(f"case {w.name} query={query}", flush=True)
        lab, core = run(ctx, x, w.eps, w.minpts)
        assert np.array_equal(core, want[1]) and np.array_equal(lab, want[0])
        ctx.close()


def test_batch_with_hashing(G):
    # instances of different d share one table; every instance's identifiers
    # carry its id above the widest coordinate fields
    rng = np.random.default_rng(41)
    problems = []
    for k in range(20):
        d = int(rng.integers(1, 5))
        n = int(rng.integers(0, 700))
        problems.append((rng.integers(0, 400, size=(n, d)).astype(np.int32), int(rng.integers(5, 40)),
                         int(rng.integers(1, 8))))
    ctx = ctx_for(G, HASH)
    ctx.set_option(G.GD_OPT_GRAPH, 0)
    outs = ctx.dbscan_batched([(torch.from_numpy(x.astype(np.float32)).cuda(), e, m) for x, e, m in problems])
    for k, ((lab, core), (x, e, m)) in enumerate(zip(outs, problems)):
        wl, wc = oracle.dbscan(x, e, m)
        assert np.array_equal(core.cpu().numpy(), wc) and np.array_equal(lab.cpu().numpy(), wl), f"instance {k}"
    ctx.close()


def test_default_order_follows_grid_size(G):
    # dense grids (H-like, about 150 points each): offset order; sparse 7-D
    # grids (about two points each): walk order; the labels are the same
    for name, n, ordered in (("H", 100_000, True), ("cfg2", 60_000, False)):
        w = W.WORKLOADS[name].with_n(n)
        x = W.make_points(w)
        ctx = G.Context(0)
        ctx.set_option(G.GD_OPT_NEIGHBOR_MODE, 1)
        lab, core = run(ctx, x, w.eps, w.minpts)
        _, gs, ids = ctx.debug_grids()
        off, nei = ctx.debug_neighbors()
        in_order = all(
            [steps.grid_offset(ids[g], ids[h]) for h in nei[off[g]:off[g + 1]]] ==
            sorted(steps.grid_offset(ids[g], ids[h]) for h in nei[off[g]:off[g + 1]])
            for g in range(0, len(ids), max(1, len(ids) // 200)))
        if ordered:
            assert in_order, name
        wl, wc = oracle.dbscan(x, w.eps, w.minpts)
        assert np.array_equal(core, wc) and np.array_equal(lab, wl)
        ctx.close()


@pytest.mark.parametrize("name,n", [("cfg2", 120_000), ("cfg1", 150_000)])
def test_walk_order_ranges_of_larger_neighbours(G, name, n):
    # walk-order lists keep each grid's larger-index neighbours in one range,
    # which is all the tiny-set merge reads: every such list splits into
    # smaller indices, then larger ones up to the range's end, then smaller
    # ones again, and the merge considers exactly the pairs it considers
    # with offset-ordered lists (filtered by index instead)
    w = W.WORKLOADS[name].with_n(n)
    x = W.make_points(w)
    want = oracle.dbscan(x, w.eps, w.minpts)
    pairs = {}
    for query in (TREE_WALK_ORDER, TREE):
        ctx = ctx_for(G, query)
        ctx.set_option(G.GD_OPT_STATS, 1)
        print(f"case {name} n={n} query={query}", flush=True)
        lab, core = run(ctx, x, w.eps, w.minpts)
        assert np.array_equal(core, want[1]) and np.array_equal(lab, want[0])
        pairs[query] = ctx.stats()["merge_pairs"]
        if query == TREE_WALK_ORDER:
            _, gs, ids = ctx.debug_grids()
            off, nei = ctx.debug_neighbors()
            for g in range(0, len(ids), max(1, len(ids) // 300)):
                lst = np.asarray(nei[off[g]:off[g + 1]], dtype=np.int64)
                above = lst > g
                if above.any():
                    first, last = np.flatnonzero(above)[[0, -1]]
                    assert above[first:last + 1].all(), f"grid {g}: larger neighbours not contiguous"
        ctx.close()
    assert pairs[TREE_WALK_ORDER] == pairs[TREE]
