"""Merge orders (GD_OPT_MERGE_ORDER): grid order with union-find, LDF
(ascending core count, Section 5.2), and the breadth-first searches of
Algorithm 6 (Section 4.4), plus the learned proposal on top of LDF.  The
components do not depend on the order (Theorem 4), so every order must give
the oracle's labels bit for bit; only the work differs."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import mlp, steps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ORDERS = {"grid": 0, "ldf": 1, "bfs": 2}


@pytest.fixture(scope="module")
def G():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G


def run(ctx, x, eps, minpts):
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    lab, core = ctx.dbscan(t, eps, minpts)
    return lab.cpu().numpy(), core.cpu().numpy()


def same(got, want, what):
    assert np.array_equal(got[1], want[1]), f"{what}: core flags differ"
    bad = np.nonzero(got[0] != want[0])[0]
    assert bad.size == 0, f"{what}: {bad.size} labels differ, first at {bad[:5]}"


@pytest.mark.parametrize("order", sorted(ORDERS))
@pytest.mark.parametrize("seed", range(8))
def test_random_vs_brute(G, order, seed):
    rng = np.random.default_rng(8000 + seed)
    d = 1 + seed % 6
    n = int(rng.integers(50, 900))
    domain = int(rng.integers(40, 400))
    x = rng.integers(0, domain, size=(n, d)).astype(np.int32)
    eps = int(rng.integers(2, max(3, domain // 5)))
    while sum(int(v).bit_length() for v in steps.cell_ids(x, eps).max(axis=0)) > 64:
        eps += 1
    minpts = int(rng.choice([1, 2, 4, 8, 20]))
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_MERGE_ORDER, ORDERS[order])
    print(f"case order={order} seed={seed} n={n} d={d} eps={eps} minpts={minpts}", flush=True)
    same(run(ctx, x, eps, minpts), oracle.dbscan_brute(x, eps, minpts), f"{order} seed {seed}")
    ctx.close()


@pytest.mark.parametrize("name,n", [("cfg1", 200_000), ("H", 200_000), ("cfg4", 200_000), ("cfg0", 10_000)])
def test_workloads_every_order(G, name, n):
    w = W.WORKLOADS[name].with_n(n)
    x = W.make_points(w)
    want = oracle.dbscan(x, w.eps, w.minpts)
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_STATS, 1)
    work = {}
    for order, v in ORDERS.items():
        ctx.set_option(G.GD_OPT_MERGE_ORDER, v)
        print(f"case {w.name} order={order}", flush=True)
        same(run(ctx, x, w.eps, w.minpts), want, f"{w.name} {order}")
        work[order] = ctx.stats()
    ctx.set_option(G.GD_OPT_MERGE_ORDER, ORDERS["ldf"])
    ctx.set_proposal(np.asarray(mlp.init(3), dtype=np.float16))
    same(run(ctx, x, w.eps, w.minpts), want, f"{w.name} learned")
    ctx.set_proposal(None)
    for order, st in work.items():
        # every considered pair is either tested or skipped
        assert st["merge_pairs"] == st["merge_tests"] + st["merge_skipped"], order
        assert st["merge_yes"] <= st["merge_tests"], order
    # each order merges the same core grids into the same components
    assert len({st["core_grids"] for st in work.values()}) == 1
    ctx.close()


def test_bfs_order_refuses_nothing_and_keeps_working(G):
    # the BFS order runs eagerly (no graph) and the context returns to LDF
    w = W.WORKLOADS["cfg1"].with_n(100_000)
    x = W.make_points(w)
    want = oracle.dbscan(x, w.eps, w.minpts)
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_GRAPH, 2)
    ctx.set_option(G.GD_OPT_MERGE_ORDER, 2)
    for _ in range(2):
        same(run(ctx, x, w.eps, w.minpts), want, "bfs with graph mode on")
        assert ctx.stats()["graph_replays"] == 0
    ctx.set_option(G.GD_OPT_LDF_ORDER, 1)
    for rep in range(2):
        same(run(ctx, x, w.eps, w.minpts), want, "ldf after bfs")
        assert ctx.stats()["graph_replays"] == rep
    ctx.close()
