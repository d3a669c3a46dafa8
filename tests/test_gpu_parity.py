"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Core flags and labels must be bit-exact (integer results); intermediate
results are checked against their definitions in oracle.steps.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import steps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    G.load_library()
    return G


@pytest.fixture(scope="module")
def ctx(G):
    c = G.Context(0)
    yield c
    c.close()


def gpu_dbscan(ctx, x, eps, minpts):
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    lab, core = ctx.dbscan(t, eps, minpts)
    return lab.cpu().numpy(), core.cpu().numpy()


@pytest.fixture()
def list_ctx(G):
    """A context that writes every grid's neighbour list out, ordered by
    offset (the debug views of Nei(g) need the lists; by default sparse data
    in d >= 4 would walk instead, and sparse grids take walk order)."""
    c = G.Context(0)
    c.set_option(G.GD_OPT_NEIGHBOR_MODE, 1)
    c.set_option(G.GD_OPT_NEIGHBOR_QUERY, 3)
    yield c
    c.close()


def assert_same(got, want, what=""):
    gl, gc = got
    wl, wc = want
    bad_c = np.nonzero(gc != wc)[0]
    bad_l = np.nonzero(gl != wl)[0]
    assert bad_c.size == 0, f"{what}: {bad_c.size} core flags differ, first at {bad_c[:5]}"
    assert bad_l.size == 0, (f"{what}: {bad_l.size} labels differ, first at {bad_l[:5]}: "
                             f"got {gl[bad_l[:5]]} want {wl[bad_l[:5]]}")


def test_handworked(ctx, golden_dir):
    with open(os.path.join(golden_dir, "handworked.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        x = np.array(c["points"], np.int32)
        lab, core = gpu_dbscan(ctx, x, c["eps"], c["minpts"])
        assert lab.tolist() == c["labels"], c["name"]
        assert core.tolist() == c["core"], c["name"]


@pytest.mark.parametrize("seed", range(24))
def test_random_small_vs_brute(ctx, seed):
    rng = np.random.default_rng(1000 + seed)
    d = 1 + seed % 8
    n = int(rng.integers(1, 700))
    domain = int(rng.integers(20, 400))
    x = rng.integers(0, domain, size=(n, d)).astype(np.int32) - domain // 3
    if n > 6:
        x[: n // 5] = x[n // 5: 2 * (n // 5)]  # duplicates
    eps = int(rng.integers(1, max(2, domain // 4)))
    while sum(int(v).bit_length() for v in steps.cell_ids(x, eps).max(axis=0)) > 128:
        eps += 1  # packed identifiers must fit two words
    minpts = int(rng.choice([1, 2, 3, 5, 9, 17, max(1, n // 3), n + 1]))
    print(f"case seed={seed} n={n} d={d} eps={eps} minpts={minpts}", flush=True)
    assert_same(gpu_dbscan(ctx, x, eps, minpts), oracle.dbscan_brute(x, eps, minpts), f"seed {seed}")


@pytest.mark.parametrize("eps,d", [(10000, 2), (10000, 3), (10000, 5), (10001, 3), (15000, 5), (21845, 2)])
def test_eps_around_packed_limit(ctx, eps, d):
    # core marking takes 16-bit coordinate differences up to eps = 10000 and
    # full words above; clusters of width 2 eps put neighbour-grid
    # differences near their bound of about 2.13 eps
    rng = np.random.default_rng(eps * 10 + d)
    n = 1500
    centres = rng.integers(0, 6 * eps, size=(8, d))
    x = (centres[rng.integers(0, 8, size=n)] + rng.integers(-eps, eps + 1, size=(n, d))).astype(np.int32)
    print(f"case eps={eps} d={d}", flush=True)
    assert_same(gpu_dbscan(ctx, x, eps, 6), oracle.dbscan_brute(x, eps, 6), f"eps {eps} d {d}")


@pytest.mark.parametrize("eps,d", [(1766, 3), (1767, 3), (134, 5), (135, 5), (33, 8), (34, 8), (21845, 2)])
def test_eps_around_packed_rows(ctx, eps, d):
    # the sorted rows are rebuilt from each coordinate's low 32 // d bits and
    # the grid while eps / sqrt(d) + 4 < 2^(32 // d), gathered above: each
    # pair straddles that bound (d = 2 fits up to the largest eps accepted);
    # points fill whole grids, edges included
    rng = np.random.default_rng(eps * 10 + d)
    n = 1500
    x = rng.integers(-3 * eps, 5 * eps, size=(n, d)).astype(np.int32)
    x[:40] = (x[:40] // eps) * eps  # on grid-aligned multiples of eps
    print(f"case eps={eps} d={d}", flush=True)
    assert_same(gpu_dbscan(ctx, x, eps, 4), oracle.dbscan_brute(x, eps, 4), f"eps {eps} d {d}")


def test_cfg0_full(ctx):
    w = W.WORKLOADS["cfg0"]
    x = W.make_points(w)
    assert_same(gpu_dbscan(ctx, x, w.eps, w.minpts), oracle.dbscan(x, w.eps, w.minpts), "cfg0")


@pytest.mark.parametrize("name,n", [("cfg1", 200_000), ("H", 200_000), ("cfg4", 300_000), ("cfg2", 100_000)])
def test_scaled_workloads(ctx, name, n):
    w = W.WORKLOADS[name].with_n(n)
    x = W.make_points(w)
    print(f"case {w.name} d={w.d} eps={w.eps} minpts={w.minpts}", flush=True)
    assert_same(gpu_dbscan(ctx, x, w.eps, w.minpts), oracle.dbscan(x, w.eps, w.minpts), w.name)


def test_grids_and_sort_match_eq1(ctx):
    rng = np.random.default_rng(7)
    for d in (1, 2, 3, 5, 8):
        x = rng.integers(-3000, 3000, size=(3000, d)).astype(np.int32)
        eps = int(rng.integers(50, 900))
        gpu_dbscan(ctx, x, eps, 4)
        sidx, gs, ids = ctx.debug_grids()
        assert np.array_equal(np.sort(sidx), np.arange(len(x)))
        want = steps.cell_ids(x, eps)
        # every point of grid g carries g's identifiers, grids are in
        # lexicographic order, input order is kept inside a grid
        for g in range(len(gs) - 1):
            members = sidx[gs[g]:gs[g + 1]]
            assert (want[members] == ids[g]).all()
            assert (np.diff(members.astype(np.int64)) > 0).all()
        assert [tuple(r) for r in ids.tolist()] == sorted(tuple(r) for r in ids.tolist())
        assert len(np.unique(want, axis=0)) == len(gs) - 1


def _grid_points(grids, side_units):
    # one point per grid at identifier * side (side chosen so Eq. (1) maps it back)
    return np.array([[k * side_units for k in g] for g in grids], np.int32)


def test_paper_grid_example(list_ctx, golden_dir):
    ctx = list_ctx
    with open(os.path.join(golden_dir, "paper_grid_example.json")) as f:
        ex = json.load(f)
    # eps = 100, d = 2: side 70.71; coordinate 71 k lands in grid k for k < 244
    x = _grid_points(ex["grids"], 71)
    gpu_dbscan(ctx, x, 100, ex["minpts"])
    sidx, gs, ids = ctx.debug_grids()
    assert ids.tolist() == ex["grids"]
    off, nei = ctx.debug_neighbors()
    q = ex["query"] - 1
    assert sorted((nei[off[q]:off[q + 1]] + 1).tolist()) == ex["nei_of_query"]


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6])
def test_neighbors_match_definition(list_ctx, d):
    ctx = list_ctx
    rng = np.random.default_rng(50 + d)
    n = 1500 if d < 5 else 800
    x = rng.integers(0, 1200, size=(n, d)).astype(np.int32)
    eps = 150
    gpu_dbscan(ctx, x, eps, 3)
    sidx, gs, ids = ctx.debug_grids()
    off, nei = ctx.debug_neighbors()
    want, woff = steps.neighbor_grids(ids)
    for g in range(len(ids)):
        got = nei[off[g]:off[g + 1]].astype(np.int64)
        assert sorted(got.tolist()) == want[g].tolist(), f"grid {g}"
        # ordered by offset (nearest grids first)
        o = [steps.grid_offset(ids[g], ids[h]) for h in got]
        assert o == sorted(o)


def test_core_flags_in_sorted_order(ctx):
    w = W.WORKLOADS["cfg1"].with_n(50_000)
    x = W.make_points(w)
    gpu_dbscan(ctx, x, w.eps, w.minpts)
    sidx, gs, ids = ctx.debug_grids()
    core_sorted, glab = ctx.debug_core()
    _, want = oracle.dbscan(x, w.eps, w.minpts)
    assert np.array_equal(core_sorted, want[sidx])


def test_merge_test_equals_min_dist(ctx):
    rng = np.random.default_rng(11)
    for eps in (10, 37, 200):
        side = eps / np.sqrt(3)
        pts, pairs, pos = [], [], 0
        want = []
        for k in range(400):
            ma, mb = int(rng.integers(1, 300)), int(rng.integers(1, 300))
            a = (rng.random((ma, 3)) * side).astype(np.int64)
            b = (rng.random((mb, 3)) * side).astype(np.int64)
            shift = int(np.ceil(side)) + int(rng.integers(0, int(1.2 * eps)))
            b[:, k % 3] += shift
            if k % 7 == 0:  # a pair exactly on the boundary: one point at distance eps
                b = np.concatenate([b, a[:1] + np.array([[eps if j == k % 3 else 0 for j in range(3)]])])
                mb += 1
            if k % 11 == 0:  # one unit beyond
                a = a[:1].repeat(3, axis=0)
                b = a[:1] + np.array([[0, 0, 0]]) + np.eye(3, dtype=np.int64)[k % 3] * (eps + 1)
                ma, mb = 3, 1
            pts += [a, b]
            pairs.append([pos, ma, pos + ma, mb])
            pos += ma + mb
            want.append(steps.min_dist2(a, b) <= eps * eps)
        P = np.concatenate(pts).T.astype(np.int32)
        ans = ctx.merge_test(torch.from_numpy(P).cuda(), torch.tensor(pairs, dtype=torch.int32).cuda(), eps)
        got = ans.cpu().numpy()
        assert (got <= 1).all()
        assert got.astype(bool).tolist() == want, f"eps {eps}"
        assert sum(want) > 20 and len(want) - sum(want) > 20


def test_ldf_order_off_gives_same_labels(ctx, G):
    w = W.WORKLOADS["H"].with_n(100_000)
    x = W.make_points(w)
    a = gpu_dbscan(ctx, x, w.eps, w.minpts)
    ctx.set_option(G.GD_OPT_LDF_ORDER, 0)
    try:
        b = gpu_dbscan(ctx, x, w.eps, w.minpts)
    finally:
        ctx.set_option(G.GD_OPT_LDF_ORDER, 1)
    assert_same(a, b, "LDF on/off")


def test_stats(ctx, G):
    w = W.WORKLOADS["cfg1"].with_n(100_000)
    x = W.make_points(w)
    ctx.set_option(G.GD_OPT_STATS, 1)
    try:
        lab, core = gpu_dbscan(ctx, x, w.eps, w.minpts)
        s = ctx.stats()
    finally:
        ctx.set_option(G.GD_OPT_STATS, 0)
    assert s["n"] == len(x) and s["core_points"] == int(core.sum())
    # every streamed candidate is tested against at least one and at most 64 open queries
    assert 0 < s["core_candidates"] <= s["core_distances"] <= 64 * s["core_candidates"]
    assert s["core_neighbor_grids"] > 0
    assert s["merge_pairs"] == s["merge_skipped"] + s["merge_tests"]
    assert 0 < s["merge_yes"] <= s["merge_tests"]
    assert s["merge_max_iterations"] >= 1


def test_error_paths(ctx, G):
    x = torch.zeros((10, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(G.GDError) as e:
        ctx.dbscan(x + 0.5, 5, 2)
    assert e.value.status == G.GD_ERANGE
    with pytest.raises(G.GDError) as e:
        ctx.dbscan(x, 1.5, 2)
    assert e.value.status == G.GD_EINVAL
    with pytest.raises(G.GDError) as e:
        ctx.dbscan(x, 0, 2)
    assert e.value.status == G.GD_EINVAL
    with pytest.raises(G.GDError) as e:
        ctx.dbscan(x, 5, 0)
    assert e.value.status == G.GD_EINVAL
    with pytest.raises(G.GDError) as e:
        ctx.dbscan(torch.zeros((4, 9), dtype=torch.float32, device="cuda"), 5, 2)
    assert e.value.status == G.GD_EINVAL
    # eps above the 32-bit distance bound is valid (64-bit distances)
    lab, core = ctx.dbscan(x, G.EPS_MAX + 1, 2)
    assert bool((core == 1).all()) and bool((lab == 0).all())
    big = torch.tensor([[0.0, 0.0], [float(1 << 25), 0.0]], device="cuda")
    with pytest.raises(G.GDError) as e:
        ctx.dbscan(big, 5, 2)
    assert e.value.status == G.GD_ERANGE
    nan = torch.tensor([[0.0, float("nan")]], device="cuda")
    with pytest.raises(G.GDError) as e:
        ctx.dbscan(nan, 5, 2)
    assert e.value.status == G.GD_ERANGE
    # identifiers wider than 128 bits: 8 dimensions spanning 2^25 with eps = 1 (about 216 bits)
    wide = torch.zeros((2, 8), dtype=torch.float32, device="cuda")
    wide[1] = float(1 << 24)
    wide[0] = -float(1 << 24)
    with pytest.raises(G.GDError) as e:
        ctx.dbscan(wide, 1, 2)
    assert e.value.status == G.GD_ERANGE
    # one grid with more core points than the merge kernels' LDS bitmaps
    # hold is valid input: one cluster, every point core
    dup = torch.zeros((270_000, 2), dtype=torch.float32, device="cuda")
    lab, core = ctx.dbscan(dup, 5, 2)
    assert bool((core == 1).all()) and bool((lab == 0).all())
    # empty input
    lab, core = ctx.dbscan(torch.zeros((0, 3), dtype=torch.float32, device="cuda"), 5, 2)
    assert lab.numel() == 0 and core.numel() == 0
    # the context still works after errors
    lab, core = ctx.dbscan(x, 1, 2)
    assert (core.cpu().numpy() == 1).all() and (lab.cpu().numpy() == 0).all()


def test_workspace_limit(G):
    c = G.Context(0)
    try:
        c.set_option(G.GD_OPT_WORKSPACE_LIMIT, 1 << 20)
        x = torch.from_numpy(W.make_points(W.WORKLOADS["cfg0"]).astype(np.float32)).cuda()
        with pytest.raises(G.GDError) as e:
            c.dbscan(x, 100, 10)
        assert e.value.status == G.GD_ENOMEM
        c.set_option(G.GD_OPT_WORKSPACE_LIMIT, 0)
        lab, core = c.dbscan(x, 100, 10)
        want = oracle.dbscan(W.make_points(W.WORKLOADS["cfg0"]), 100, 10)
        assert_same((lab.cpu().numpy(), core.cpu().numpy()), want, "after limit")
    finally:
        c.close()


def test_repeat_and_shuffle(ctx):
    w = W.WORKLOADS["cfg0"]
    x = W.make_points(w)
    a = gpu_dbscan(ctx, x, w.eps, w.minpts)
    b = gpu_dbscan(ctx, x, w.eps, w.minpts)
    assert_same(a, b, "repeat")
    perm = np.random.default_rng(3).permutation(len(x))
    xs = x[perm]
    assert_same(gpu_dbscan(ctx, xs, w.eps, w.minpts), oracle.dbscan(xs, w.eps, w.minpts), "shuffled")
