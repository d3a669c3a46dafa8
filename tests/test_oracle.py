"""Pins for the CPU oracle: every check compares it with something that is
not itself -- hand-worked examples, brute force, closed forms, special
cases that reduce to library routines, and invariants."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W


def _canon(labels):
    """Relabel clusters by first appearance so partitions compare as sets."""
    out = np.full(labels.shape, -1, np.int64)
    seen = {}
    for i, l in enumerate(labels):
        if l < 0:
            continue
        out[i] = seen.setdefault(int(l), len(seen))
    return out


def _brute_pairs(x):
    x = x.astype(np.int64)
    diff = x[:, None, :] - x[None, :, :]
    return (diff * diff).sum(axis=2)


def test_handworked_examples(golden_dir):
    with open(os.path.join(golden_dir, "handworked.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        x = np.array(c["points"], np.int32)
        for fn in (oracle.dbscan, oracle.dbscan_brute):
            labels, core = fn(x, c["eps"], c["minpts"])
            assert labels.tolist() == c["labels"], (c["name"], fn.__name__)
            assert core.tolist() == c["core"], (c["name"], fn.__name__)


@pytest.mark.parametrize("seed", range(40))
def test_grid_oracle_equals_brute_force(seed):
    rng = np.random.default_rng(seed)
    d = int(rng.integers(1, 6))
    n = int(rng.integers(0, 300))
    domain = int(rng.integers(5, 200))
    x = rng.integers(0, domain, size=(n, d)).astype(np.int32)
    if n > 4:  # duplicates
        x[: n // 4] = x[n // 4: 2 * (n // 4)]
    eps = int(rng.integers(1, max(2, domain // 3)))
    minpts = int(rng.choice([1, 2, 3, 5, 8, max(1, n), n + 1]))
    lg, cg = oracle.dbscan(x, eps, minpts)
    lb, cb = oracle.dbscan_brute(x, eps, minpts)
    assert np.array_equal(cg, cb)
    assert np.array_equal(lg, lb)


def test_ties_on_the_sphere():
    # squared distance exactly eps^2 is a neighbour, eps^2 + 1 is not (closed ball)
    eps = 5
    x = np.array([[0, 0], [3, 4], [0, 5], [5, 1], [40, 40]], np.int32)  # 25, 25, 26
    D = _brute_pairs(x)
    assert D[0, 1] == 25 and D[0, 2] == 25 and D[0, 3] == 26
    labels, core = oracle.dbscan(x, eps, 3)
    # p0 sees p0, p1, p2 -> core; p1 sees p0,p1,p2(9+1=10),p3(4+9=13) -> core
    assert core.tolist()[:2] == [1, 1]
    lb, cb = oracle.dbscan_brute(x, eps, 3)
    assert np.array_equal(labels, lb) and np.array_equal(core, cb)


@pytest.mark.parametrize("seed", range(6))
def test_matches_scikit_learn(seed):
    from sklearn.cluster import DBSCAN
    rng = np.random.default_rng(100 + seed)
    d = int(rng.integers(2, 5))
    x = W.random_small(seed, 3000, d, 1000)
    eps, minpts = int(rng.integers(20, 80)), int(rng.integers(3, 15))
    labels, core = oracle.dbscan(x, eps, minpts)
    m = DBSCAN(eps=eps, min_samples=minpts, algorithm="kd_tree").fit(x.astype(np.float64))
    sk_core = np.zeros(len(x), bool)
    sk_core[m.core_sample_indices_] = True
    assert np.array_equal(sk_core, core.astype(bool))
    # same partition of the core points
    cm = core.astype(bool)
    assert np.array_equal(_canon(labels[cm]), _canon(m.labels_[cm]))
    # same border set (sklearn may give a border point another valid cluster)
    assert np.array_equal(labels[~cm] >= 0, m.labels_[~cm] >= 0)


def test_cfg0_matches_scikit_learn_and_brute():
    from sklearn.cluster import DBSCAN
    w = W.WORKLOADS["cfg0"]
    x = W.make_points(w)
    labels, core = oracle.dbscan(x, w.eps, w.minpts)
    lb, cb = oracle.dbscan_brute(x, w.eps, w.minpts)
    assert np.array_equal(labels, lb) and np.array_equal(core, cb)
    m = DBSCAN(eps=w.eps, min_samples=w.minpts, algorithm="kd_tree").fit(x.astype(np.float64))
    cm = core.astype(bool)
    assert np.array_equal(np.isin(np.arange(len(x)), m.core_sample_indices_), cm)
    assert np.array_equal(_canon(labels[cm]), _canon(m.labels_[cm]))


@pytest.mark.parametrize("seed", range(5))
def test_minpts_one_is_connected_components(seed):
    # MinPts = 1: every point is core and clusters are the connected
    # components of the eps-graph (scipy's routine).
    from scipy.sparse.csgraph import connected_components
    from sklearn.neighbors import radius_neighbors_graph
    d = 1 + seed % 4
    x = W.random_small(200 + seed, 1500, d, 3000)
    eps = 60
    labels, core = oracle.dbscan(x, eps, 1)
    assert core.all()
    g = radius_neighbors_graph(x.astype(np.float64), eps, mode="connectivity", include_self=True)
    ncomp, comp = connected_components(g, directed=False)
    # canonical id of a component = its smallest index
    first = np.full(ncomp, len(x))
    np.minimum.at(first, comp, np.arange(len(x)))
    assert np.array_equal(labels, first[comp])


@pytest.mark.parametrize("seed", range(5))
def test_one_dimension_closed_form(seed):
    # d = 1: sort; |N(p)| is a window count (searchsorted); two core points
    # are connected iff every gap between consecutive core points between
    # them is <= eps.
    rng = np.random.default_rng(300 + seed)
    n = 2000
    x = rng.integers(0, 20000, size=(n, 1)).astype(np.int32)
    eps, minpts = int(rng.integers(3, 30)), int(rng.integers(2, 8))
    v = x[:, 0].astype(np.int64)
    s = np.sort(v)
    cnt = np.searchsorted(s, v + eps, side="right") - np.searchsorted(s, v - eps, side="left")
    core = cnt >= minpts
    order = np.argsort(v, kind="stable")
    cv = [i for i in order if core[i]]
    comp = {}
    cid = -1
    prev = None
    for i in cv:
        if prev is None or v[i] - v[prev] > eps:
            cid += 1
        comp[i] = cid
        prev = i
    cmin = {}
    for i, c in comp.items():
        cmin[c] = min(cmin.get(c, i), i)
    expect = np.full(n, -1, np.int64)
    for i, c in comp.items():
        expect[i] = cmin[c]
    core_idx = np.array(sorted(comp))
    for i in range(n):
        if core[i]:
            continue
        near = core_idx[np.abs(v[core_idx] - v[i]) <= eps]
        if near.size:
            expect[i] = cmin[comp[int(near.min())]]
    labels, ocore = oracle.dbscan(x, eps, minpts)
    assert np.array_equal(ocore.astype(bool), core)
    assert np.array_equal(labels, expect)


def test_degenerate_cases():
    x = W.random_small(7, 500, 3, 100)
    # MinPts > n: nobody is core, everything is noise
    labels, core = oracle.dbscan(x, 10, 501)
    assert not core.any() and (labels == -1).all()
    # eps beyond the diameter: one cluster with every point core, id 0
    labels, core = oracle.dbscan(x, 1000, 500)
    assert core.all() and (labels == 0).all()
    # empty input
    labels, core = oracle.dbscan(np.zeros((0, 2), np.int32), 5, 3)
    assert labels.shape == (0,) and core.shape == (0,)
    # a single point
    labels, core = oracle.dbscan(np.array([[5, 5]], np.int32), 5, 1)
    assert labels.tolist() == [0] and core.tolist() == [1]
    labels, core = oracle.dbscan(np.array([[5, 5]], np.int32), 5, 2)
    assert labels.tolist() == [-1] and core.tolist() == [0]
    # all points identical
    labels, core = oracle.dbscan(np.zeros((50, 4), np.int32), 1, 50)
    assert core.all() and (labels == 0).all()


@pytest.mark.parametrize("seed", range(4))
def test_invariants(seed):
    # core <=> |N| >= MinPts; core points within eps share a label; each
    # cluster is connected through core points; a border point is within eps
    # of a core point of its cluster, namely its lowest-index core neighbour;
    # a noise point has no core neighbour; ids are the clusters' smallest core
    # index.
    rng = np.random.default_rng(400 + seed)
    d = int(rng.integers(2, 4))
    x = W.make_points(W.WORKLOADS["cfg0"].with_n(2500)) if d == 2 else W.random_small(seed, 2500, d, 600)
    eps, minpts = (100, 10) if d == 2 else (40, 6)
    labels, core = oracle.dbscan(x, eps, minpts)
    D = _brute_pairs(x)
    nb = D <= eps * eps
    cnt = nb.sum(axis=1)
    assert np.array_equal(core.astype(bool), cnt >= minpts)
    cm = core.astype(bool)
    ci = np.nonzero(cm)[0]
    sub = nb[np.ix_(ci, ci)]
    a, b = np.nonzero(sub)
    assert np.array_equal(labels[ci[a]], labels[ci[b]])
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    ncomp, comp = connected_components(csr_matrix(sub), directed=False)
    assert ncomp == len(np.unique(labels[ci]))
    for k in range(ncomp):
        members = ci[comp == k]
        assert (labels[members] == members.min()).all()
    for i in np.nonzero(~cm)[0]:
        cn = ci[nb[i, ci]]
        if cn.size == 0:
            assert labels[i] == -1
        else:
            assert labels[i] == labels[cn.min()]


def test_neighbor_count_brute_agrees_with_core_flags():
    w = W.WORKLOADS["cfg1"]
    x = W.make_points(w, n=20000)
    labels, core = oracle.dbscan(x, w.eps, w.minpts)
    q = np.arange(0, 20000, 37)
    cnt = oracle.neighbor_count_brute(x, w.eps, q)
    assert np.array_equal(cnt >= w.minpts, core[q].astype(bool))
    xi = x.astype(np.int64)
    for k in q[:20]:
        direct = (((xi - xi[k]) ** 2).sum(axis=1) <= w.eps ** 2).sum()
        assert cnt[list(q).index(k)] == direct


def test_rejects_bad_arguments():
    x = np.zeros((3, 2), np.int32)
    with pytest.raises(ValueError):
        oracle.dbscan(x.astype(np.float32) + 0.5, 1, 1)
    with pytest.raises(ValueError):
        oracle.dbscan(x, 0, 1)
    with pytest.raises(RuntimeError):
        oracle.dbscan(x, 1, 0)
    with pytest.raises(RuntimeError):
        oracle.dbscan(np.full((2, 2), 1 << 25, np.int32), 1, 1)
