"""Launch tunables (points per workgroup, waves per FastMerging workgroup)
and the autotuner: every configuration must give exactly the oracle's
result, and the autotuner must keep one of the timed configurations."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ws = W.batch_workloads(count=10, seed_base=4242)
    problems = [(W.make_points(w, n=min(w.n, 20_000)), w.eps, w.minpts) for w in ws]
    refs = [oracle.dbscan(x, e, m) for x, e, m in problems]
    dev = [(torch.from_numpy(x.astype(np.float32)).cuda(), e, m) for x, e, m in problems]
    return G, problems, refs, dev


@pytest.mark.parametrize("tile", [256, 1024, 8192])
@pytest.mark.parametrize("waves", [1, 2, 4])
def test_every_configuration_is_exact(setup, tile, waves):
    G, problems, refs, dev = setup
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_TILE_POINTS, tile)
    ctx.set_option(G.GD_OPT_MERGE_WAVES, waves)
    print(f"case: tile {tile}, merge waves {waves}", flush=True)
    outs = ctx.dbscan_batched(dev)
    for k, ((lab, core), (wl, wc)) in enumerate(zip(outs, refs)):
        assert np.array_equal(core.cpu().numpy(), wc), f"instance {k}: core flags differ"
        assert np.array_equal(lab.cpu().numpy(), wl), f"instance {k}: labels differ"
    ctx.close()


def test_bad_tunables_are_rejected(setup):
    G = setup[0]
    ctx = G.Context(0)
    for opt, val in ((G.GD_OPT_TILE_POINTS, 100), (G.GD_OPT_TILE_POINTS, 0), (G.GD_OPT_MERGE_WAVES, 3)):
        with pytest.raises(G.GDError):
            ctx.set_option(opt, val)
    ctx.close()


def test_autotune_keeps_a_timed_configuration(setup):
    G, problems, refs, dev = setup
    ctx = G.Context(0)
    best, rows = ctx.autotune(dev)
    assert len(rows) == 12
    assert all(r["ms"] > 0 for r in rows)
    assert best == {k: min(rows, key=lambda r: r["ms"])[k] for k in ("tile_points", "merge_waves")}
    # the tuned context still gives the exact result, also through graph replay
    for rep in range(2):
        outs = ctx.dbscan_batched(dev)
        for k, ((lab, core), (wl, wc)) in enumerate(zip(outs, refs)):
            assert np.array_equal(core.cpu().numpy(), wc) and np.array_equal(lab.cpu().numpy(), wl)
    ctx.close()
