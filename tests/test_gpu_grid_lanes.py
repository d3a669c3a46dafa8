"""Lanes per grid in the tiny-core-set merge (GD_OPT_GRID_LANES): four grids
per wave or one.  The result must not depend on it, and must be the
oracle's."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


@pytest.mark.parametrize("lanes", [16, 64])
@pytest.mark.parametrize("seed", range(6))
def test_random_vs_brute(G, lanes, seed):
    rng = np.random.default_rng(4400 + seed)
    d = 1 + seed % 5
    n = int(rng.integers(1, 900))
    x = rng.integers(0, 300, size=(n, d)).astype(np.int32)
    eps = int(rng.integers(3, 40))
    minpts = int(rng.choice([1, 2, 3, 5]))
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_GRID_LANES, lanes)
    ctx.set_option(G.GD_OPT_STATS, 1)
    print(f"case lanes={lanes} seed={seed} n={n} d={d} eps={eps} minpts={minpts}", flush=True)
    lab, core = run(ctx, x, eps, minpts)
    wl, wc = oracle.dbscan_brute(x, eps, minpts)
    assert np.array_equal(core, wc) and np.array_equal(lab, wl)
    st = ctx.stats()
    assert st["merge_pairs"] == st["merge_tests"] + st["merge_skipped"]
    ctx.close()


@pytest.mark.parametrize("name,n", [("cfg0", 10_000), ("cfg2", 100_000), ("H", 100_000)])
def test_workloads_every_lane_count(G, name, n):
    w = W.WORKLOADS[name].with_n(n)
    x = W.make_points(w)
    want = oracle.dbscan(x, w.eps, w.minpts)
    for lanes in (0, 16, 64):
        ctx = G.Context(0)
        ctx.set_option(G.GD_OPT_GRID_LANES, lanes)
        print(f"case {w.name} lanes={lanes}", flush=True)
        lab, core = run(ctx, x, w.eps, w.minpts)
        assert np.array_equal(core, want[1]) and np.array_equal(lab, want[0])
        ctx.close()


def test_batch_prefix_and_replay(G):
    ws = W.batch_workloads()[:24]
    probs = [(W.make_points(w.with_n(min(w.n, 40_000))), w.eps, w.minpts) for w in ws]
    want = [oracle.dbscan(x, e, m) for x, e, m in probs]
    tens = [(torch.from_numpy(x.astype(np.float32)).cuda(), e, m) for x, e, m in probs]
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_GRID_LANES, 16)
    for rep in range(3):
        outs = ctx.dbscan_batched(tens)
        assert ctx.stats()["graph_replays"] == (1 if rep else 0)
        for k, ((lab, core), (wl, wc)) in enumerate(zip(outs, want)):
            assert np.array_equal(core.cpu().numpy(), wc) and np.array_equal(lab.cpu().numpy(), wl), f"instance {k}"
    with pytest.raises(G.GDError):
        ctx.set_option(G.GD_OPT_GRID_LANES, 8)
    ctx.close()
