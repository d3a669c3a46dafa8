"""Walk mode (GD_OPT_NEIGHBOR_MODE = 2): core marking, the merging of tiny
core sets and border assignment walk the grid tree for their own grid
instead of reading neighbour lists written out first.  The result must be
bit-exact against the oracle and equal to list mode, on every dimension, with
tiny and large core sets mixed, in batches, under graph replay and with the
learned proposal on."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import steps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LISTS, WALKS = 1, 2


@pytest.fixture(scope="module")
def G():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G


@pytest.fixture(scope="module")
def walk_ctx(G):
    c = G.Context(0)
    c.set_option(G.GD_OPT_NEIGHBOR_MODE, WALKS)
    yield c
    c.close()


def run(ctx, x, eps, minpts):
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    lab, core = ctx.dbscan(t, eps, minpts)
    return lab.cpu().numpy(), core.cpu().numpy()


def assert_same(got, want, what):
    gl, gc = got
    wl, wc = want
    bad_c = np.nonzero(gc != wc)[0]
    bad_l = np.nonzero(gl != wl)[0]
    assert bad_c.size == 0, f"{what}: {bad_c.size} core flags differ, first at {bad_c[:5]}"
    assert bad_l.size == 0, (f"{what}: {bad_l.size} labels differ, first at {bad_l[:5]}: "
                             f"got {gl[bad_l[:5]]} want {wl[bad_l[:5]]}")


@pytest.mark.parametrize("seed", range(24))
def test_random_small_vs_brute(walk_ctx, seed):
    rng = np.random.default_rng(5000 + seed)
    d = 1 + seed % 8
    n = int(rng.integers(1, 700))
    domain = int(rng.integers(20, 400))
    x = rng.integers(0, domain, size=(n, d)).astype(np.int32) - domain // 3
    if n > 6:
        x[: n // 5] = x[n // 5: 2 * (n // 5)]  # duplicates
    eps = int(rng.integers(1, max(2, domain // 4)))
    while sum(int(v).bit_length() for v in steps.cell_ids(x, eps).max(axis=0)) > 128:
        eps += 1
    minpts = int(rng.choice([1, 2, 3, 5, 9, 17, max(1, n // 3), n + 1]))
    print(f"case seed={seed} n={n} d={d} eps={eps} minpts={minpts}", flush=True)
    got = run(walk_ctx, x, eps, minpts)
    assert walk_ctx.stats()["neighbor_walk"] == 1
    assert_same(got, oracle.dbscan_brute(x, eps, minpts), f"seed {seed}")


@pytest.mark.parametrize("d", [2, 3, 5, 8])
def test_tiny_and_large_core_sets_mixed(walk_ctx, d):
    # dense clumps (core sets far above 8 points, merged from lists) beside
    # sparse chains (tiny core sets, merged by the walks) that touch them
    rng = np.random.default_rng(77 + d)
    eps = 40
    clumps = [rng.integers(0, 600, size=d) + rng.integers(-8, 9, size=(60, d)) for _ in range(6)]
    chain = np.cumsum(rng.integers(-9, 10, size=(700, d)), axis=0) + 300
    noise = rng.integers(-200, 900, size=(300, d))
    x = np.concatenate(clumps + [chain, noise]).astype(np.int32)
    x = x[rng.permutation(len(x))]
    print(f"case mixed d={d} n={len(x)}", flush=True)
    for minpts in (3, 6, 12):
        assert_same(run(walk_ctx, x, eps, minpts), oracle.dbscan_brute(x, eps, minpts), f"d {d} minpts {minpts}")


@pytest.mark.parametrize("name,n", [("cfg0", 10_000), ("cfg1", 150_000), ("H", 100_000), ("cfg2", 300_000),
                                    ("cfg4", 150_000)])
def test_workloads_vs_oracle_and_lists(G, walk_ctx, name, n):
    w = W.WORKLOADS[name].with_n(n)
    x = W.make_points(w)
    print(f"case {w.name} d={w.d} eps={w.eps} minpts={w.minpts}", flush=True)
    got = run(walk_ctx, x, w.eps, w.minpts)
    assert_same(got, oracle.dbscan(x, w.eps, w.minpts), w.name)
    lists = G.Context(0)
    lists.set_option(G.GD_OPT_NEIGHBOR_MODE, LISTS)
    assert_same(got, run(lists, x, w.eps, w.minpts), f"{w.name}: walk vs lists")
    assert lists.stats()["neighbor_walk"] == 0
    lists.close()


def test_auto_mode_walks_when_lists_do_not_fit(G):
    # by default every grid gets its list; when the lists would not fit the
    # workspace (here the fixed array of dbscan_noalloc: sparse 5-D data with
    # hundreds of neighbours per grid) the consumers walk the grid tree
    ctx = G.Context(0)
    w = W.WORKLOADS["cfg2"].with_n(450_000)
    x = W.make_points(w)
    want = oracle.dbscan(x, w.eps, w.minpts)
    print(f"case {w.name} auto mode", flush=True)
    got = run(ctx, x, w.eps, w.minpts)
    st = ctx.stats()
    assert st["neighbor_walk"] == 0
    assert st["neighbor_entries"] * 4 > G.NOALLOC_SCRATCH_BYTES // 2  # beside the workspace they do not fit
    assert_same(got, want, w.name)
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    lab = torch.empty(len(x), dtype=torch.int32, device="cuda")
    core = torch.empty(len(x), dtype=torch.uint8, device="cuda")
    ctx.dbscan_noalloc(t, w.eps, w.minpts, lab, core)
    assert ctx.stats()["neighbor_walk"] == 1
    assert_same((lab.cpu().numpy(), core.cpu().numpy()), want, f"{w.name} in the fixed array")
    ctx.close()


def test_stats_in_walk_mode(G, walk_ctx):
    w = W.WORKLOADS["cfg2"].with_n(200_000)
    x = W.make_points(w)
    walk_ctx.set_option(G.GD_OPT_STATS, 1)
    try:
        got = run(walk_ctx, x, w.eps, w.minpts)
        st = walk_ctx.stats()
    finally:
        walk_ctx.set_option(G.GD_OPT_STATS, 0)
    assert_same(got, oracle.dbscan(x, w.eps, w.minpts), "stats run")
    assert st["neighbor_walk"] == 1 and st["merge_tests"] > 0 and st["core_distances"] > 0
    assert st["merge_pairs"] == st["merge_tests"] + st["merge_skipped"]
    with pytest.raises(G.GDError) as e:
        walk_ctx.debug_neighbors()
    assert e.value.status == G.GD_EUNSUPPORTED


def test_batched_walk_mode(G, walk_ctx):
    rng = np.random.default_rng(91)
    problems = []
    for k in range(30):
        d = int(rng.integers(1, 7))
        n = int(rng.integers(0, 900))
        x = rng.integers(0, 500, size=(n, d)).astype(np.int32)
        problems.append((x, int(rng.integers(5, 60)), int(rng.integers(1, 12))))
    print("case: 30 random instances in walk mode", flush=True)
    walk_ctx.set_option(G.GD_OPT_GRAPH, 0)
    try:
        outs = walk_ctx.dbscan_batched([(torch.from_numpy(x.astype(np.float32)).cuda(), e, m)
                                        for x, e, m in problems])
    finally:
        walk_ctx.set_option(G.GD_OPT_GRAPH, 1)
    for k, ((lab, core), (x, e, m)) in enumerate(zip(outs, problems)):
        assert_same((lab.cpu().numpy(), core.cpu().numpy()), oracle.dbscan(x, e, m), f"instance {k}")


def test_graph_replay_in_walk_mode(G):
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_NEIGHBOR_MODE, WALKS)
    ctx.set_option(G.GD_OPT_GRAPH, 2)
    w = W.WORKLOADS["cfg2"].with_n(150_000)
    x = W.make_points(w)
    want = oracle.dbscan(x, w.eps, w.minpts)
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    for rep in range(4):
        print(f"case: walk-mode call {rep}", flush=True)
        lab, core = ctx.dbscan(t, w.eps, w.minpts)
        st = ctx.stats()
        assert st["graph_replays"] == (1 if rep else 0) and st["neighbor_walk"] == 1
        assert_same((lab.cpu().numpy(), core.cpu().numpy()), want, f"call {rep}")
    ctx.close()


def test_proposal_in_walk_mode(G, walk_ctx):
    from oracle import mlp
    w = W.WORKLOADS["cfg4"].with_n(120_000)
    x = W.make_points(w)
    want = oracle.dbscan(x, w.eps, w.minpts)
    walk_ctx.set_proposal(np.asarray(mlp.init(7), dtype=np.float16))
    try:
        got = run(walk_ctx, x, w.eps, w.minpts)
    finally:
        walk_ctx.set_proposal(None)
    assert_same(got, want, "proposal on, walk mode")
