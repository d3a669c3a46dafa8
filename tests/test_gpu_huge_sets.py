"""Core sets larger than the merge kernels' LDS bitmaps (more than 262144
core points in one grid), and heavy ones (8192 or more) that eager calls
merge with a workgroup per pair.  The pairs with such a set are queued and
tested with bitmaps in device memory; the result must be DBSCAN's, also in
graph replays (which test heavy sets on one wave each).

The point sets are built so that the clustering follows from distances
alone (the oracle's pair scan would take hours on them): boxes whose
diameter is below eps are all core, and the gaps between boxes decide which
clusters join.  Small and tiny core sets and a border point sit beside the
oversized ones so that every kind of pair meets them."""
import numpy as np
import pytest

import oracle
from oracle import steps

torch = pytest.importorskip("torch")

EPS, MINPTS = 100, 5
BIG = 300_000


def boxes(seed, scale=1, big=BIG):
    """Points and their cluster by construction (-1: noise; the border point
    gets the cluster of its core neighbours), for eps = 100 * scale."""
    rng = np.random.default_rng(seed)

    def box(m, x0, x1, y0, y1):
        return np.stack([rng.integers(x0 * scale, x1 * scale + 1, m), rng.integers(y0 * scale, y1 * scale + 1, m)],
                        axis=1)

    parts = [
        (box(big, 0, 40, 0, 40), 0),          # A
        (box(big, 81, 121, 0, 40), 0),        # B: 41 from A
        (box(big, 230, 270, 0, 40), 1),       # C: 109 from B, apart
        (box(50, 300, 310, 0, 10), 1),        # D: a small set inside C's reach
        (np.array([[-50, 0], [-50, 1], [-50, 2]]) * scale, 0),   # E: tiny core set next to A
        (np.array([[-140, 0]]) * scale, 0),   # border: 90 from E, 4 neighbours with itself
        (np.array([[20_000 + 1000 * k, 5000] for k in range(10)]) * scale, -1),  # noise
    ]
    x = np.concatenate([p for p, _ in parts]).astype(np.int32)
    cl = np.concatenate([np.full(len(p), c) for p, c in parts])
    perm = rng.permutation(len(x))
    return np.ascontiguousarray(x[perm]), cl[perm]


def expected(x, cl, scale=1):
    """Canonical labels: a cluster's id is its smallest core index; the
    border point (the only non-core point of a cluster) takes its cluster's."""
    border = np.nonzero((x[:, 0] == -140 * scale) & (x[:, 1] == 0))[0]
    core = (cl >= 0).astype(np.uint8)
    core[border] = 0
    lab = np.full(len(x), -1, np.int64)
    for c in (0, 1):
        idx = np.nonzero((cl == c) & (core == 1))[0]
        lab[cl == c] = idx.min()
    return lab.astype(np.int32), core


@pytest.fixture(scope="module")
def G():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G


@pytest.fixture(scope="module")
def data():
    x, cl = boxes(3)
    ids = steps.cell_ids(x, EPS)
    _, counts = np.unique(ids, axis=0, return_counts=True)
    assert counts.max() > 262_144  # the construction does produce oversized grids
    return x, expected(x, cl)


def run(ctx, x):
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    lab, core = ctx.dbscan(t, EPS, MINPTS)
    return lab.cpu().numpy(), core.cpu().numpy()


@pytest.mark.parametrize("seed,scale", [(3, 1), (4, 300)])
def test_construction_pinned_on_a_sample(seed, scale):
    # the same recipe, boxes thinned out so the oracle's pair scan is quick:
    # the clusters must be the ones the construction names
    x, cl = boxes(seed, scale)
    keep = np.zeros(len(x), bool)
    rng = np.random.default_rng(0)
    for c in (0, 1):
        idx = np.nonzero(cl == c)[0]
        keep[rng.choice(idx, size=min(len(idx), 4000), replace=False)] = True
    keep[(x[:, 0] <= -50 * scale) | (x[:, 0] >= 300 * scale)] = True  # every E, D, border and noise point
    xs, cs = x[keep], cl[keep]
    lab, core = oracle.dbscan(xs, EPS * scale, MINPTS)
    want_l, want_c = expected(xs, cs, scale)
    assert np.array_equal(core, want_c) and np.array_equal(lab, want_l)


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["ldf", "grid_order", "bfs", "walk"])
def test_oversized_core_sets(G, data, mode):
    x, (want_l, want_c) = data
    ctx = G.Context(0)
    if mode == "grid_order":
        ctx.set_option(G.GD_OPT_LDF_ORDER, 0)
    elif mode == "bfs":
        ctx.set_option(G.GD_OPT_MERGE_ORDER, 2)
    elif mode == "walk":
        ctx.set_option(G.GD_OPT_NEIGHBOR_MODE, 2)
    ctx.set_option(G.GD_OPT_STATS, 1)
    print(f"case oversized core sets, {mode}", flush=True)
    lab, core = run(ctx, x)
    st = ctx.stats()
    assert np.array_equal(core, want_c)
    bad = np.nonzero(lab != want_l)[0]
    assert bad.size == 0, f"{bad.size} labels differ, first at {bad[:5]}"
    assert st["merge_pairs"] == st["merge_tests"] + st["merge_skipped"]
    assert st["merge_yes"] >= 1
    ctx.close()


@pytest.mark.gpu
def test_oversized_core_sets_run_eagerly_in_graph_mode(G, data):
    x, (want_l, want_c) = data
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_GRAPH, 2)
    for rep in range(3):
        print(f"case graph mode call {rep}", flush=True)
        lab, core = run(ctx, x)
        assert ctx.stats()["graph_replays"] == 0
        assert np.array_equal(core, want_c) and np.array_equal(lab, want_l)
    # a small input afterwards captures and replays as usual
    small = np.ascontiguousarray(x[np.abs(x[:, 0]) > 10_000])
    for rep in range(3):
        run(ctx, small)
        assert ctx.stats()["graph_replays"] == (1 if rep else 0)
    ctx.close()


@pytest.mark.gpu
def test_oversized_core_sets_without_allocation(G, data):
    x, (want_l, want_c) = data
    ctx = G.Context(0)
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    lab = torch.empty(len(x), dtype=torch.int32, device="cuda")
    core = torch.empty(len(x), dtype=torch.uint8, device="cuda")
    print("case oversized core sets through dbscan_noalloc", flush=True)
    ctx.dbscan_noalloc(t, EPS, MINPTS, lab, core)
    assert np.array_equal(core.cpu().numpy(), want_c) and np.array_equal(lab.cpu().numpy(), want_l)
    ctx.close()


@pytest.mark.gpu
@pytest.mark.parametrize("order", [1, 2])
def test_oversized_core_sets_with_wide_distances(G, order):
    # the same construction at eps = 30000, above the 32-bit distance bound
    scale = 300
    x, cl = boxes(4, scale)
    ids = steps.cell_ids(x, EPS * scale)
    _, counts = np.unique(ids, axis=0, return_counts=True)
    assert counts.max() > 262_144
    want_l, want_c = expected(x, cl, scale)
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_MERGE_ORDER, order)
    print(f"case oversized core sets, eps {EPS * scale}, order {order}", flush=True)
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    lab, core = ctx.dbscan(t, EPS * scale, MINPTS)
    assert np.array_equal(core.cpu().numpy(), want_c) and np.array_equal(lab.cpu().numpy(), want_l)
    ctx.close()


@pytest.mark.gpu
@pytest.mark.parametrize("mode", ["ldf", "bfs", "grid_order"])
def test_heavy_core_sets(G, mode):
    # 20000-point boxes: heavy (merged by a workgroup per pair in eager
    # calls) but within the LDS bitmaps (one wave per pair in replays)
    x, cl = boxes(5, 1, 20_000)
    _, counts = np.unique(steps.cell_ids(x, EPS), axis=0, return_counts=True)
    assert 8192 <= counts.max() <= 262_144
    want_l, want_c = expected(x, cl)
    ctx = G.Context(0)
    if mode == "bfs":
        ctx.set_option(G.GD_OPT_MERGE_ORDER, 2)
    elif mode == "grid_order":
        ctx.set_option(G.GD_OPT_LDF_ORDER, 0)
    ctx.set_option(G.GD_OPT_STATS, 1)
    print(f"case heavy core sets, {mode}", flush=True)
    lab, core = run(ctx, x)
    st = ctx.stats()
    assert np.array_equal(core, want_c) and np.array_equal(lab, want_l)
    assert st["merge_pairs"] == st["merge_tests"] + st["merge_skipped"]
    ctx.set_option(G.GD_OPT_STATS, 0)
    if mode == "ldf":
        ctx.set_option(G.GD_OPT_GRAPH, 2)
        for rep in range(3):
            lab, core = run(ctx, x)
            assert ctx.stats()["graph_replays"] == (1 if rep else 0)
            assert np.array_equal(core, want_c) and np.array_equal(lab, want_l)
    ctx.close()
