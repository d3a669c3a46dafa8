"""Pins for the oracle's step definitions: Eq. (1) identifiers, the
neighbouring-grid rule of Algorithm 3, the worked grid example of Section
4.1-4.2, the merge test of Definition 6 / Theorem 2 and the step model of
Algorithm 5."""
import decimal
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import steps


def test_cell_ids_against_high_precision_division():
    # floor((p - mn) / (eps / sqrt(d))) in 60-digit decimal arithmetic
    decimal.getcontext().prec = 60
    rng = np.random.default_rng(1)
    for _ in range(300):
        d = int(rng.integers(1, 9))
        eps = int(rng.integers(1, 20000))
        x = rng.integers(-(1 << 24), (1 << 24) + 1, size=(4, d)).astype(np.int64)
        ids = steps.cell_ids(x, eps)
        mn = x.min(axis=0)
        side = decimal.Decimal(eps) / decimal.Decimal(d).sqrt()
        for i in range(4):
            for j in range(d):
                want = int((decimal.Decimal(int(x[i, j] - mn[j])) / side).to_integral_value(decimal.ROUND_FLOOR))
                assert ids[i, j] == want


def test_cell_ids_on_exact_boundaries():
    # d = 4: sqrt(d) = 2, so u = k * eps / 2 sits exactly on a boundary
    eps = 10
    x = np.array([[0, 0, 0, 0], [5, 4, 15, 14], [10, 9, 20, 19]], np.int64)
    ids = steps.cell_ids(x, eps)
    assert ids.tolist() == [[0, 0, 0, 0], [1, 0, 3, 2], [2, 1, 4, 3]]


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5])
def test_candidate_offset_counts_closed_form(d):
    # Per coordinate, max(|v|-1,0)^2 is 0 for three values, 1 for two, 4 for
    # two, 9 for two, ...  Count vectors whose sum stays below d by choosing
    # how many coordinates take each nonzero contribution.
    contrib = [(0, 3)] + [(k * k, 2) for k in range(1, d + 1)]
    # dynamic programme over coordinates on the total contribution
    ways = {0: 1}
    for _ in range(d):
        nxt = {}
        for tot, w in ways.items():
            for c, mult in contrib:
                if tot + c < d:
                    nxt[tot + c] = nxt.get(tot + c, 0) + w * mult
        ways = nxt
    closed = sum(ways.values())
    assert closed == {1: 3, 2: 21, 3: 117, 4: 609, 5: 3903}[d]
    assert len(steps.candidate_offsets(d)) == closed


def test_paper_grid_example(golden_dir):
    with open(os.path.join(golden_dir, "paper_grid_example.json")) as f:
        ex = json.load(f)
    grids = np.array(ex["grids"])
    nei, offs = steps.neighbor_grids(grids)
    q = ex["query"] - 1
    assert sorted((nei[q] + 1).tolist()) == ex["nei_of_query"]
    # grids are already in the lexicographic order of Section 4.1
    assert [tuple(g) for g in grids] == sorted(tuple(g) for g in grids)
    # first level of the query: root children with key within ceil(sqrt(2)) = 2
    keys = sorted(set(grids[:, 0].tolist()))
    c = math.ceil(math.sqrt(ex["d"]))
    assert [k for k in keys if abs(k - grids[q, 0]) <= c] == ex["first_level_keys_of_query"]
    # t4 = grid (1,1) reached through t3 (key 1): offset 1 + 1 = 2 >= d
    assert steps.grid_offset((1, 1), grids[q]) == ex["t4_offset"]
    assert grids.max() == ex["eta"]


@pytest.mark.parametrize("seed", range(6))
def test_same_grid_within_eps_and_neighbours_cover_eps(seed):
    # P1: two points in one grid are within eps; P2: two points within eps
    # lie in the same grid or in grids whose offset is below d.
    rng = np.random.default_rng(seed)
    d = int(rng.integers(1, 6))
    eps = int(rng.integers(3, 40))
    x = rng.integers(0, 6 * eps, size=(400, d)).astype(np.int64)
    ids = steps.cell_ids(x, eps)
    diff = x[:, None, :] - x[None, :, :]
    D = (diff * diff).sum(axis=2)
    gd = np.abs(ids[:, None, :] - ids[None, :, :])
    off = (np.maximum(gd - 1, 0) ** 2).sum(axis=2)
    same = (gd == 0).all(axis=2)
    assert (D[same] < eps * eps).all()
    assert (off[D <= eps * eps] < d).all()
    assert (gd[D <= eps * eps] <= math.ceil(math.sqrt(d))).all()


def test_neighbor_grids_match_candidate_enumeration():
    x = W.make_points(W.WORKLOADS["cfg0"].with_n(3000))
    cells, counts, _ = steps.cell_assignment(x, 100)
    nei, _ = steps.neighbor_grids(cells)
    index = {tuple(c): i for i, c in enumerate(cells.tolist())}
    cand = [v for v in steps.candidate_offsets(2) if any(v)]
    for i, c in enumerate(cells.tolist()):
        want = sorted(index[t] for t in (tuple(a + b for a, b in zip(c, v)) for v in cand) if t in index)
        assert nei[i].tolist() == want


def _merge_cases(rng, m):
    for _ in range(m):
        d = int(rng.integers(2, 5))
        eps = int(rng.integers(5, 40))
        side = eps / math.sqrt(d)
        # two grids one above the other along dimension 0, with a random gap
        a = (rng.random((int(rng.integers(1, 40)), d)) * side).astype(np.int64)
        b = (rng.random((int(rng.integers(1, 40)), d)) * side).astype(np.int64)
        b[:, 0] += int(math.ceil(side)) + int(rng.integers(0, 2 * eps))
        yield a, b, eps


def test_fast_merging_equals_min_dist():
    rng = np.random.default_rng(5)
    n_yes = n_no = 0
    for a, b, eps in _merge_cases(rng, 1500):
        ans, iters, evals = steps.fast_merging(a, b, eps)
        assert ans == steps.can_merge(a, b, eps)
        n_yes += ans
        n_no += not ans
        assert evals <= iters * 3 * (len(a) + len(b))
    assert n_yes > 100 and n_no > 100


def test_fast_merging_boundary_ties():
    eps = 5
    a = np.array([[0, 0], [0, 1], [1, 0]])
    # exactly eps away: merge; one unit further: no merge
    assert steps.fast_merging(a, np.array([[1, 5], [9, 9]]), eps)[0] is True
    assert steps.fast_merging(a, np.array([[0, 7], [9, 9]]), eps)[0] is False
    # squared distance eps^2 + 1
    assert steps.fast_merging(np.array([[0, 0]]), np.array([[1, 5]]), eps)[0] is False
    # duplicates across the sets
    assert steps.fast_merging(np.array([[3, 3]] * 5), np.array([[3, 3]]), eps)[0] is True
    # collinear far points
    assert steps.fast_merging(np.array([[i, 0] for i in range(5)]), np.array([[i, 0] for i in range(11, 20)]), eps)[0] is False


def test_fast_merging_distance_tally():
    # one full iteration that ends in 'no' after both prunings: r1 + 3 r2 + 2 r1'
    a = np.array([[0, 0]])
    b = np.array([[0, 20], [0, 21]])
    ans, iters, evals = steps.fast_merging(a, b, 5)
    assert ans is False and iters == 1
    # s_i = {p} is emptied by the first Pruning: r2 (nearest) + r1 + r2 (Pruning)
    assert evals == 2 + 1 + 2
    a = np.array([[0, 0], [0, 1]])
    b = np.array([[0, 20], [30, 30]])
    ans, iters, evals = steps.fast_merging(a, b, 5)
    assert ans is False


def test_fast_merging_terminates_without_angle_rule():
    # every half iteration drops the probe point itself (triangle rule with
    # dist(x, p) = 0 < sigma), so iterations never exceed the set sizes
    rng = np.random.default_rng(9)
    for a, b, eps in _merge_cases(rng, 300):
        ans, iters, _ = steps.fast_merging(a, b, eps)
        assert iters <= min(len(a), len(b))
