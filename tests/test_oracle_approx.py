"""Pins for oracle.core_components, the bound the approximate merge is
checked against."""
import numpy as np

import oracle
import workloads as W


def test_radius_eps_is_dbscan_partition_of_core_points():
    for seed in range(6):
        rng = np.random.default_rng(seed)
        d = 1 + seed % 4
        x = rng.integers(0, 300, size=(400, d)).astype(np.int32)
        eps, minpts = 20, 4
        lab, core = oracle.dbscan_brute(x, eps, minpts)
        comp = oracle.core_components(x, core, eps)
        assert np.array_equal(comp[core == 1], lab[core == 1])
        assert np.all(comp[core == 0] == -1)


def test_gap_between_clumps_joins_only_within_eps_plus_delta():
    # two clumps whose nearest points are 12 apart: separate at eps 10,
    # one component at 10 + 2 (the closed bound) and above
    a = np.array([[0, 0], [3, 0], [6, 0], [9, 0]], np.int32)
    b = a + np.array([21, 0], np.int32)
    x = np.concatenate([a, b])
    core = np.ones(len(x), np.uint8)
    assert len(set(oracle.core_components(x, core, 10).tolist())) == 2
    assert len(set(oracle.core_components(x, core, 11).tolist())) == 2
    assert set(oracle.core_components(x, core, 12).tolist()) == {0}


def test_labels_are_smallest_core_index():
    x = W.random_small(3, 300, 2, 200)
    core = np.zeros(300, np.uint8)
    core[::3] = 1
    lab = oracle.core_components(x, core, 30)
    for v in set(lab[lab >= 0].tolist()):
        members = np.nonzero(lab == v)[0]
        assert v == members.min() and core[v] == 1
