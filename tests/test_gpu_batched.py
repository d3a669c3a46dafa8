"""Batched clustering: many instances of uneven n, d, eps and MinPts in one
pass of the pipeline.  Every instance must get exactly the oracle's result
(and the single-instance call's result)."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = G.Context(0)
    yield c
    c.close()


def _check(outs, problems):
    for k, ((lab, core), (x, eps, minpts)) in enumerate(zip(outs, problems)):
        wl, wc = oracle.dbscan(x, eps, minpts)
        gl, gc = lab.cpu().numpy(), core.cpu().numpy()
        assert np.array_equal(gc, wc), f"instance {k}: core flags differ"
        assert np.array_equal(gl, wl), f"instance {k}: labels differ"


def test_small_mixed_batch(ctx):
    rng = np.random.default_rng(77)
    problems = []
    for k in range(40):
        d = int(rng.integers(1, 6))
        n = int(rng.integers(0, 900))
        x = rng.integers(0, 500, size=(n, d)).astype(np.int32)
        eps = int(rng.integers(5, 60))
        minpts = int(rng.integers(1, 12))
        problems.append((x, eps, minpts))
    print(f"case: 40 random instances, d in 1..5", flush=True)
    outs = ctx.dbscan_batched([(torch.from_numpy(x.astype(np.float32)).cuda(), e, m) for x, e, m in problems])
    _check(outs, problems)


def test_batch_workload_prefix(ctx):
    # the first 24 instances of the 256-instance batch workload, capped in size
    ws = W.batch_workloads()[:24]
    problems = [(W.make_points(w, n=min(w.n, 60_000)), w.eps, w.minpts) for w in ws]
    print(f"case: batch prefix, total n = {sum(len(p[0]) for p in problems)}", flush=True)
    outs = ctx.dbscan_batched([(torch.from_numpy(x.astype(np.float32)).cuda(), e, m) for x, e, m in problems])
    _check(outs, problems)


def test_batch_equals_single_calls(ctx):
    ws = W.batch_workloads()[24:40]
    problems = [(W.make_points(w, n=min(w.n, 40_000)), w.eps, w.minpts) for w in ws]
    tens = [(torch.from_numpy(x.astype(np.float32)).cuda(), e, m) for x, e, m in problems]
    outs = ctx.dbscan_batched(tens)
    for (lab, core), (t, e, m) in zip(outs, tens):
        l1, c1 = ctx.dbscan(t, e, m)
        assert torch.equal(lab, l1) and torch.equal(core, c1)


def test_batch_errors(ctx):
    import paper_2210_07580_amd as G
    good = torch.zeros((5, 2), dtype=torch.float32, device="cuda")
    bad = good + 0.25
    with pytest.raises(G.GDError) as e:
        ctx.dbscan_batched([(good, 3, 2), (bad, 3, 2)])
    assert e.value.status == G.GD_ERANGE and "instance 1" in str(e.value)
    with pytest.raises(G.GDError) as e:
        ctx.dbscan_batched([(good, 3, 2), (good, 2.5, 2)])
    assert e.value.status == G.GD_EINVAL
    assert ctx.dbscan_batched([]) == []
    outs = ctx.dbscan_batched([(good, 3, 2), (torch.zeros((0, 3), dtype=torch.float32, device="cuda"), 3, 2)])
    assert (outs[0][1].cpu().numpy() == 1).all() and outs[1][0].numel() == 0


def test_full_batch_workload_matches_oracle_digests(ctx):
    """All 256 instances of the batch workload at full size (sum of n about
    34M), in one dbscan_batched() call as the benchmark makes it, against the
    oracle's per-instance digests (tests/golden/make_oracle_digests.py cfg3),
    then once more replayed from the captured graph."""
    import hashlib
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_digests.json")
    with open(path) as f:
        recs = json.load(f).get("cfg3")
    if recs is None:
        pytest.skip("no stored oracle digests for the batch workload")

    def sha(a):
        return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()

    ws = W.batch_workloads()
    assert len(recs) == len(ws)
    probs = []
    for k, (w, rec) in enumerate(zip(ws, recs)):
        x = W.make_points(w)
        assert sha(x) == rec["points_sha256"], f"instance {k}: generator output changed"
        probs.append((torch.from_numpy(x.astype(np.float32)).cuda(), w.eps, w.minpts))
    print(f"case: full batch workload, {len(probs)} instances, "
          f"{sum(int(p[0].shape[0]) for p in probs)} points", flush=True)
    for rep in range(2):
        outs = ctx.dbscan_batched(probs)
        assert ctx.stats()["graph_replays"] == rep
        for k, ((lab, core), rec) in enumerate(zip(outs, recs)):
            assert sha(core.cpu().numpy().astype(np.uint8)) == rec["core_sha256"], f"instance {k}: core flags"
            assert sha(lab.cpu().numpy().astype("<i4")) == rec["labels_sha256"], f"instance {k}: labels"


def test_batch_mixing_every_dimension(ctx):
    """One batch holding instances of every d from 1 to 8 (the kernels run
    for d = 8, shorter rows padded), eagerly, replayed from a graph, and with
    the consumers walking the tree: every instance must be the oracle's."""
    rng = np.random.default_rng(123)
    problems = []
    for k in range(24):
        d = k % 8 + 1
        n = int(rng.integers(1, 3000))
        centres = rng.integers(0, 4000, size=(max(1, n // 60), d))
        x = (centres[rng.integers(0, len(centres), size=n)] + rng.integers(-90, 91, size=(n, d))).astype(np.int32)
        x[: n // 10] = rng.integers(0, 4000, size=(n // 10, d))
        problems.append((x, int(rng.integers(20, 120)), int(rng.integers(2, 12))))
    tens = [(torch.from_numpy(x.astype(np.float32)).cuda(), e, m) for x, e, m in problems]
    for graph, mode in ((1, 0), (0, 2)):
        import paper_2210_07580_amd as G
        c = G.Context(0)
        c.set_option(G.GD_OPT_GRAPH, graph)
        c.set_option(G.GD_OPT_NEIGHBOR_MODE, mode)
        for rep in range(2 if graph else 1):
            print(f"case: d 1..8 batch, graph {graph} mode {mode} call {rep}", flush=True)
            _check(c.dbscan_batched(tens), problems)
            if graph:
                assert c.stats()["graph_replays"] == rep
        c.close()
