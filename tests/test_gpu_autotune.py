"""Launch tunables (points per workgroup, waves per FastMerging workgroup,
lanes per small grid) and the autotuner: every configuration must give
exactly the oracle's result, the autotuner must keep one of the timed
configurations, and its tuning file must hand the choice to a new context
without timing anything."""
import json

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
@pytest.mark.parametrize("lanes", [16, 64])
def test_every_configuration_is_exact(setup, tile, waves, lanes):
    G, problems, refs, dev = setup
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_TILE_POINTS, tile)
    ctx.set_option(G.GD_OPT_MERGE_WAVES, waves)
    ctx.set_option(G.GD_OPT_GRID_LANES, lanes)
    print(f"case: tile {tile}, merge waves {waves}, lanes {lanes}", flush=True)
    outs = ctx.dbscan_batched(dev)
    for k, ((lab, core), (wl, wc)) in enumerate(zip(outs, refs)):
        assert np.array_equal(core.cpu().numpy(), wc), f"instance {k}: core flags differ"
        assert np.array_equal(lab.cpu().numpy(), wl), f"instance {k}: labels differ"
    ctx.close()


def test_bad_tunables_are_rejected(setup):
    G = setup[0]
    ctx = G.Context(0)
    for opt, val in ((G.GD_OPT_TILE_POINTS, 100), (G.GD_OPT_TILE_POINTS, 0), (G.GD_OPT_MERGE_WAVES, 3),
                     (G.GD_OPT_GRID_LANES, 32)):
        with pytest.raises(G.GDError):
            ctx.set_option(opt, val)
    ctx.close()


def test_autotune_keeps_a_timed_configuration(setup):
    G, problems, refs, dev = setup
    ctx = G.Context(0)
    best, rows = ctx.autotune(dev)
    assert len(rows) == 12
    assert all(r["ms"] > 0 for r in rows)
    assert {(r["tile_points"], r["merge_waves"], r["grid_lanes"]) for r in rows} == {
        (t, w, l) for t in (1024, 4096) for w in (1, 2, 4) for l in (16, 64)}
    assert best == {k: min(rows, key=lambda r: r["ms"])[k] for k in ("tile_points", "merge_waves", "grid_lanes")}
    # the tuned context still gives the exact result, also through graph replay
    for rep in range(2):
        outs = ctx.dbscan_batched(dev)
        for k, ((lab, core), (wl, wc)) in enumerate(zip(outs, refs)):
            assert np.array_equal(core.cpu().numpy(), wc) and np.array_equal(lab.cpu().numpy(), wl)
    ctx.close()


def test_tuning_file_round_trip(setup, tmp_path):
    G, problems, refs, dev = setup
    path = tmp_path / "tuning.json"
    ctx = G.Context(0)
    ctx.set_tuning_file(str(path))
    best, rows = ctx.autotune(dev)
    assert len(rows) == 12
    stored = json.loads(path.read_text())
    assert len(stored) == 1
    (key, entry), = stored.items()
    assert key.startswith("count=10;")
    assert {k: entry[k] for k in best} == best
    ctx.close()
    # a new context applies the stored choice without timing, and stays exact
    ctx = G.Context(0)
    ctx.set_tuning_file(str(path))
    again, rows = ctx.autotune(dev)
    assert again is None and rows == []
    outs = ctx.dbscan_batched(dev)
    for k, ((lab, core), (wl, wc)) in enumerate(zip(outs, refs)):
        assert np.array_equal(core.cpu().numpy(), wc) and np.array_equal(lab.cpu().numpy(), wl)
    # another batch shape is searched and added beside the first
    best2, rows2 = ctx.autotune(dev[:4])
    assert len(rows2) == 12 and len(json.loads(path.read_text())) == 2
    # an unreadable file is ignored (searched again) and rewritten
    path.write_text("not json")
    _, rows3 = ctx.autotune(dev)
    assert len(rows3) == 12 and len(json.loads(path.read_text())) == 1
    ctx.close()
