"""Graph replay of batched calls: the first call for a batch shape runs with
host synchronisation and captures a synchronisation-free run into a HIP
graph; later calls of that shape replay it.  Every replay must give exactly
the eager result, with eager work and synchronisations in between, for new
coordinates of the same shape, and must fall back to an exact eager run when
the data outgrow the captured sizes."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture()
def G():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G


def _problems(seed, count=12, scale=1):
    ws = W.batch_workloads(count=count, seed_base=seed)
    out = []
    for w in ws:
        x = W.make_points(w, n=min(w.n, 30_000)) * scale
        out.append((x.astype(np.int32), w.eps, w.minpts))
    return out


def _dev(problems):
    return [(torch.from_numpy(x.astype(np.float32)).cuda(), e, m) for x, e, m in problems]


def _eager(G, problems):
    c = G.Context(0)
    c.set_option(G.GD_OPT_GRAPH, 0)
    outs = [tuple(t.cpu().numpy() for t in o) for o in c.dbscan_batched(_dev(problems))]
    assert c.stats()["graph_replays"] == 0
    c.close()
    return outs


def _same(outs, ref, what):
    for k, ((lab, core), (rl, rc)) in enumerate(zip(outs, ref)):
        assert np.array_equal(core.cpu().numpy(), rc), f"{what}: instance {k} core flags differ"
        assert np.array_equal(lab.cpu().numpy(), rl), f"{what}: instance {k} labels differ"


def test_replays_match_eager(G):
    probs = _problems(5151)
    ref = _eager(G, probs)
    # the eager reference itself against the oracle, for two instances
    for k in (0, 5):
        wl, wc = oracle.dbscan(*probs[k])
        assert np.array_equal(ref[k][0], wl) and np.array_equal(ref[k][1], wc)
    ctx = G.Context(0)
    dev = _dev(probs)
    print("case: first call (eager + capture)", flush=True)
    outs = ctx.dbscan_batched(dev)
    assert ctx.stats()["graph_replays"] == 0
    _same(outs, ref, "first call")
    other = W.make_points(W.WORKLOADS["cfg0"])
    other_t = torch.from_numpy(other.astype(np.float32)).cuda()
    for rep in range(4):
        print(f"case: replay {rep}", flush=True)
        outs = ctx.dbscan_batched(dev)
        assert ctx.stats()["graph_replays"] == 1, "the call did not replay the graph"
        _same(outs, ref, f"replay {rep}")
        # eager work of the program between replays
        lab, core = ctx.dbscan(other_t, 100, 10)
        torch.cuda.synchronize()
        assert int(core.sum().item()) > 0
    ctx.close()


def test_replay_with_new_data_of_same_shape(G):
    a = _problems(6161)
    # same instance sizes and dimensions, other coordinates, eps and MinPts
    b = []
    rng = np.random.default_rng(3)
    for x, e, m in a:
        y = rng.integers(0, 10_000, size=x.shape).astype(np.int32)
        b.append((y, int(rng.integers(60, 300)), int(rng.integers(3, 30))))
    ref_b = _eager(G, b)
    ctx = G.Context(0)
    ctx.dbscan_batched(_dev(a))  # capture on a
    print("case: replay on new data of the same shape", flush=True)
    outs = ctx.dbscan_batched(_dev(b))
    _same(outs, ref_b, "replay on new data")
    ctx.close()


def test_overflow_falls_back_exactly(G):
    a = _problems(7171)
    # same shape, but a far larger spread: many more grids than were captured
    b = [(np.random.default_rng(k).integers(0, 2_000_000, size=x.shape).astype(np.int32), 50, 3)
         for k, (x, e, m) in enumerate(a)]
    ref_b = _eager(G, b)
    ctx = G.Context(0)
    ctx.dbscan_batched(_dev(a))
    print("case: replay that outgrows the plan", flush=True)
    outs = ctx.dbscan_batched(_dev(b))
    assert ctx.stats()["graph_replays"] == 0, "an overflowing replay must rerun eagerly"
    _same(outs, ref_b, "fallback")
    # the next call of this shape captured anew and replays
    outs = ctx.dbscan_batched(_dev(b))
    assert ctx.stats()["graph_replays"] == 1
    _same(outs, ref_b, "replay after recapture")
    ctx.close()


def test_bad_input_in_replay_is_reported(G):
    a = _problems(8181, count=4)
    ctx = G.Context(0)
    ctx.dbscan_batched(_dev(a))
    bad = [(x.astype(np.float32), e, m) for x, e, m in a]
    bad[2][0][0, 0] = 0.5
    print("case: replay with a non-integer coordinate", flush=True)
    with pytest.raises(G.GDError, match="instance 2"):
        ctx.dbscan_batched([(torch.from_numpy(x).cuda(), e, m) for x, e, m in bad])
    # and the context still works
    outs = ctx.dbscan_batched(_dev(a))
    _same(outs, _eager(G, a), "after the error")
    ctx.close()


def test_single_call_graph_mode(G):
    w = W.WORKLOADS["cfg1"]
    x = W.make_points(w, n=200_000)
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    c0 = G.Context(0)
    c0.set_option(G.GD_OPT_GRAPH, 0)
    rl, rc = (v.cpu().numpy() for v in c0.dbscan(t, w.eps, w.minpts))
    c0.close()
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_GRAPH, 2)
    for rep in range(3):
        print(f"case: single-instance call {rep}", flush=True)
        lab, core = ctx.dbscan(t, w.eps, w.minpts)
        assert ctx.stats()["graph_replays"] == (1 if rep else 0)
        assert np.array_equal(core.cpu().numpy(), rc) and np.array_equal(lab.cpu().numpy(), rl)
    ctx.close()


def test_replay_with_eps_beyond_packed_rows(G):
    # Captured where each coordinate's low bits ride through the sort (d = 3,
    # eps 200: grid side 115 < 2^10); replayed with eps 2400 (side 1386), for
    # which they do not: the replay must notice, be discarded, and rerun
    # eagerly with the gather, giving the eager result.
    w = W.WORKLOADS["cfg1"]
    x = W.make_points(w, n=100_000)
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    big = 2400
    c0 = G.Context(0)
    c0.set_option(G.GD_OPT_GRAPH, 0)
    rl, rc = (v.cpu().numpy() for v in c0.dbscan(t, big, w.minpts))
    c0.close()
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_GRAPH, 2)
    ctx.dbscan(t, w.eps, w.minpts)
    ctx.dbscan(t, w.eps, w.minpts)
    assert ctx.stats()["graph_replays"] == 1
    print("case: replay with eps beyond the packed rows", flush=True)
    lab, core = ctx.dbscan(t, big, w.minpts)
    assert ctx.stats()["graph_replays"] == 0, "the replay must be discarded"
    assert np.array_equal(core.cpu().numpy(), rc) and np.array_equal(lab.cpu().numpy(), rl)
    ctx.close()


def _wrap_trap():
    """d = 2 points where a 16-bit coordinate difference wraps into the eps
    ball: point 0 sits at x = 0, five points at x = 45000 lie two grids
    away (grid side eps / sqrt(2) ~ 15447 for eps = 21845, so the grids are
    neighbours by Eq. (2)), 45000 - 2^16 = -20536 would pass |dx| <= eps.
    The true distance is 45000 > eps: point 0 is noise for MinPts 3."""
    pts = [(0, 0)] + [(45000, k) for k in range(5)] + [(90000 + 7 * k, 3 * k) for k in range(6)]
    return np.array(pts, dtype=np.int32)


def test_replay_across_packed_difference_bound(G):
    # captured at eps <= 10000 (core marking compares packed 16-bit
    # differences), then the same shape at eps 21845, where those would wrap
    x = _wrap_trap()
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    want_l, want_c = oracle.dbscan(x, 21845, 3)
    assert want_c[0] == 0 and want_l[0] == -1
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_GRAPH, 2)
    for _ in range(2):
        ctx.dbscan(t, 5000, 3)
    assert ctx.stats()["graph_replays"] == 1
    for rep, eps in enumerate((21845, 21100, 21845)):
        print(f"case: same shape at eps {eps} after a capture at eps 5000 ({rep})", flush=True)
        wl, wc = oracle.dbscan(x, eps, 3)
        lab, core = ctx.dbscan(t, eps, 3)
        assert np.array_equal(core.cpu().numpy(), wc) and np.array_equal(lab.cpu().numpy(), wl)
    # and back below the bound: the small-eps graph is captured again
    for _ in range(2):
        lab, core = ctx.dbscan(t, 5000, 3)
    wl, wc = oracle.dbscan(x, 5000, 3)
    assert np.array_equal(core.cpu().numpy(), wc) and np.array_equal(lab.cpu().numpy(), wl)
    ctx.close()


def test_instance_table_growth_drops_graph(G):
    # a graph captured for 8 instances reads the instance table through the
    # pointers of that time; a later call with more instances than the table
    # holds (one that does not capture: statistics on) reallocates it, and
    # the next call of the first shape must not replay the stale graph
    small = _problems(9191, count=8)
    many = _problems(9292, count=20)
    ctx = G.Context(0)
    outs = ctx.dbscan_batched(_dev(small))  # eager + capture
    outs = ctx.dbscan_batched(_dev(small))
    assert ctx.stats()["graph_replays"] == 1
    ctx.set_option(G.GD_OPT_STATS, 1)
    print("case: 20 instances with statistics on (instance table grows)", flush=True)
    ctx.dbscan_batched(_dev(many))
    ctx.set_option(G.GD_OPT_STATS, 0)
    print("case: the 8-instance shape again", flush=True)
    outs = ctx.dbscan_batched(_dev(small))
    assert ctx.stats()["graph_replays"] == 0, "a graph over the old instance table must not replay"
    for k, (lab, core) in enumerate(outs):
        wl, wc = oracle.dbscan(*small[k])
        assert np.array_equal(core.cpu().numpy(), wc) and np.array_equal(lab.cpu().numpy(), wl), f"instance {k}"
    outs = ctx.dbscan_batched(_dev(small))
    assert ctx.stats()["graph_replays"] == 1
    ctx.close()


def test_capturing_call_keeps_its_stats(G):
    """The call that captures a graph reports the sizes of its own eager run
    (grids, neighbour entries, core counts), as a call without graphs does,
    and so does the replay after it."""
    x, eps, minpts = _problems(71, count=1)[0]
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    plain = G.Context(0)
    plain.dbscan(t, eps, minpts)
    want = plain.stats()
    plain.close()
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_GRAPH, 2)
    for rep in range(2):
        ctx.dbscan(t, eps, minpts)
        st = ctx.stats()
        print(f"case call {rep}: grids {st['grids']} replays {st['graph_replays']}", flush=True)
        for k in ("n", "grids", "neighbor_entries", "core_points", "core_grids", "dense_grids", "key_bits"):
            assert st[k] == want[k], (rep, k, st[k], want[k])
        assert st["graph_replays"] == rep
    # the debug views describe eager calls only
    with pytest.raises(G.GDError):
        ctx.debug_grids()
    ctx.close()
