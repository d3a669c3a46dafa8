"""Approximate FastMerging (GD_OPT_APPROX_DELTA, Section 4.3.3): "yes" once a
pair within eps + delta is met.  Core flags and the border rule are exact;
the clusters must lie between DBSCAN's (eps) and the components of the core
points' (eps + delta)-graph, with canonical labels.  delta = 0 is exact."""
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


def refines(fine, coarse, mask):
    """Every class of `fine` (over mask) lies inside one class of `coarse`."""
    f, c = fine[mask], coarse[mask]
    order = np.argsort(f, kind="stable")
    f, c = f[order], c[order]
    starts = np.r_[True, f[1:] != f[:-1]]
    first = np.maximum.accumulate(np.where(starts, np.arange(len(f)), 0))
    return bool(np.all(c == c[first]))


def check_sandwich(x, eps, minpts, delta, got):
    lab, core = got
    want_l, want_c = oracle.dbscan(x, eps, minpts)
    assert np.array_equal(core, want_c), "core flags must stay exact"
    cm = want_c == 1
    relaxed = oracle.core_components(x, want_c, eps + delta)
    assert refines(want_l, lab, cm), "an exact cluster was split"
    assert refines(lab, relaxed, cm), "core points joined beyond eps + delta"
    # canonical: a cluster's label is its smallest core index
    for v in np.unique(lab[cm]):
        members = np.nonzero(cm & (lab == v))[0]
        assert members.min() == v
    # border points take the approximate label of their exact cluster; noise stays noise
    border = (~cm) & (want_l >= 0)
    assert np.all(lab[(~cm) & (want_l < 0)] == -1)
    if border.any():
        rep = {int(v): int(lab[int(v)]) for v in np.unique(want_l[border])}  # the exact cluster's id is a core index
        assert np.array_equal(lab[border], np.array([rep[int(v)] for v in want_l[border]]))


@pytest.mark.parametrize("seed", range(8))
def test_random_sandwich(G, seed):
    rng = np.random.default_rng(300 + seed)
    d = 2 + seed % 4
    n = int(rng.integers(300, 3000))
    x = rng.integers(0, 2000, size=(n, d)).astype(np.int32)
    eps = int(rng.integers(40, 160))
    minpts = int(rng.integers(2, 8))
    ctx = G.Context(0)
    for delta in (0, eps // 4, eps):
        ctx.set_option(G.GD_OPT_APPROX_DELTA, delta)
        print(f"case seed={seed} d={d} n={n} eps={eps} minpts={minpts} delta={delta}", flush=True)
        got = run(ctx, x, eps, minpts)
        if delta == 0:
            wl, wc = oracle.dbscan(x, eps, minpts)
            assert np.array_equal(got[1], wc) and np.array_equal(got[0], wl)
        check_sandwich(x, eps, minpts, delta, got)
    ctx.close()


# sizes and deltas keep the oracle's pair count (every core pair within
# eps + delta) near 1e7: the seed-spreader clumps are dense
@pytest.mark.parametrize("name,n,deltas", [("cfg1", 5_000, (20,)), ("H", 5_000, (20,)), ("cfg2", 50_000, (500, 5000)),
                                          ("cfg0", 10_000, (10, 100))])
def test_workloads_sandwich(G, name, n, deltas):
    w = W.WORKLOADS[name].with_n(n)
    x = W.make_points(w)
    ctx = G.Context(0)
    for delta in deltas:
        ctx.set_option(G.GD_OPT_APPROX_DELTA, delta)
        for order in (1, 2):
            ctx.set_option(G.GD_OPT_MERGE_ORDER, order)
            print(f"case {w.name} delta={delta} order={order}", flush=True)
            check_sandwich(x, w.eps, w.minpts, delta, run(ctx, x, w.eps, w.minpts))
    ctx.close()


def test_gap_merged_only_with_delta(G):
    # two dense clumps 12 apart (nearest points): eps 10 keeps them apart and
    # so does delta 1 (no pair within 11); with delta 50 every pair of the two
    # clumps (at most 32 apart) is within eps + delta, so the first probe
    # answers yes.  (A delta between, such as 2, may or may not join them:
    # only pairs the search meets count.)
    a = np.array([[i, j] for i in range(0, 10, 3) for j in range(0, 10, 3)], np.int32)
    b = a + np.array([21, 0], np.int32)
    x = np.concatenate([a, b])
    ctx = G.Context(0)
    for delta, parts in ((0, 2), (1, 2), (50, 1)):
        ctx.set_option(G.GD_OPT_APPROX_DELTA, delta)
        lab, core = run(ctx, x, 10, 3)
        assert core.all() and len(set(lab.tolist())) == parts, (delta, lab)
    with pytest.raises(G.GDError):
        ctx.set_option(G.GD_OPT_APPROX_DELTA, -1)
    ctx.close()
