"""Definitions of the intermediate results of grid DBSCAN.  TEST
INFRASTRUCTURE ONLY (part of the oracle; the GPU library never imports it).

Each function writes out the plain definition that the GPU path must
reproduce exactly, citing where the paper states it.  Nothing here is
blocked, fused or reordered beyond the definition.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


# --------------------------------------------------------------------------
# Eq. (1): grid identifiers.
# --------------------------------------------------------------------------
def cell_ids(points, eps: int) -> np.ndarray:
    """g_ij = floor((p_j - mn_j) / (eps / sqrt(d))), mn_j = min over P (Eq. (1)).

    Evaluated exactly for integer coordinates and integer eps: with
    u = p_j - mn_j >= 0, u / (eps / sqrt(d)) = sqrt(d u^2) / eps, and for a
    positive integer eps, floor(y / eps) = floor(floor(y) / eps), so
    g = isqrt(d u^2) // eps.  Python integers keep every step exact.
    """
    x = np.asarray(points, dtype=np.int64)
    n, d = x.shape
    if n == 0:
        return np.zeros((0, d), np.int64)
    u = x - x.min(axis=0)
    out = np.empty_like(u)
    flat_u = u.ravel()
    flat_o = out.ravel()
    for i in range(flat_u.shape[0]):
        v = int(flat_u[i])
        flat_o[i] = math.isqrt(d * v * v) // int(eps)
    return out


def nonempty_grids(ids: np.ndarray):
    """Gs: the distinct identifiers in lexicographic order (dimension 1 most
    significant, Section 4.1), with the number of points in each."""
    if ids.shape[0] == 0:
        return np.zeros((0, ids.shape[1]), np.int64), np.zeros(0, np.int64)
    cells, counts = np.unique(ids, axis=0, return_counts=True)
    return cells, counts


# --------------------------------------------------------------------------
# Neighbouring grids (Section 4.2.2, Eq. (2), Algorithm 3).
# --------------------------------------------------------------------------
def grid_offset(a, b) -> int:
    """offset(g, g') = sum_j max(|g'_j - g_j| - 1, 0)^2: the squared minimum
    distance between the two grids in units of (eps / sqrt(d))^2."""
    return int(sum(max(abs(int(p) - int(q)) - 1, 0) ** 2 for p, q in zip(a, b)))


def neighbor_grids(cells: np.ndarray):
    """Nei(g) for each non-empty grid: the non-empty grids g' != g whose
    offset is below d (Algorithm 3 drops a node once its offset reaches d).
    Returned as a list (one entry per row of ``cells``) of sorted index
    arrays, and a parallel list of offsets.  Brute force over all pairs."""
    cells = np.asarray(cells, dtype=np.int64)
    m, d = cells.shape
    out, offs = [], []
    for i in range(m):
        delta = np.abs(cells - cells[i])
        off = (np.maximum(delta - 1, 0) ** 2).sum(axis=1)
        sel = np.nonzero(off < d)[0]
        sel = sel[sel != i]
        out.append(sel)
        offs.append(off[sel])
    return out, offs


def candidate_offsets(d: int):
    """All integer offset vectors v with sum_j max(|v_j| - 1, 0)^2 < d (the
    zero vector included); |v_j| <= ceil(sqrt(d)) for each of them."""
    c = math.isqrt(d - 1) + 1 if d > 1 else 1   # ceil(sqrt(d))
    out = []
    for v in itertools.product(range(-c, c + 1), repeat=d):
        if sum(max(abs(t) - 1, 0) ** 2 for t in v) < d:
            out.append(v)
    return out


# --------------------------------------------------------------------------
# Definition 6 and Theorem 2: the merge test.
# --------------------------------------------------------------------------
def sqdist(a, b) -> int:
    return int(sum((int(p) - int(q)) ** 2 for p, q in zip(a, b)))


def min_dist2(si, sj) -> int:
    """MinDist(s_i, s_j)^2 by brute force over all pairs (Definition 6)."""
    a = np.asarray(si, dtype=np.int64)
    b = np.asarray(sj, dtype=np.int64)
    diff = a[:, None, :] - b[None, :, :]
    return int((diff * diff).sum(axis=2).min())


def can_merge(si, sj, eps: int) -> bool:
    """Two core grids merge iff MinDist of their core points <= eps
    (the merge definition of Section 3.2; Theorem 2 says FastMerging
    decides exactly this)."""
    return min_dist2(si, sj) <= int(eps) ** 2


def fast_merging(si, sj, eps: int, start: int = 0):
    """Algorithm 5 (with Algorithm 4 for Pruning), step by step in the
    paper's order, on integer points.

    Distances are compared exactly in integers.  The triangle rule keeps
    its strict '<' and the angle rule its strict 'lambda < theta'; the
    angles are evaluated in float64 as the paper writes them, and a point
    is dropped by the angle rule only with a margin of 1e-9 rad, so
    rounding can only keep a point, never drop one wrongly.  If a Pruning
    call empties a set the answer is 'no' at once (the listing's loop test
    comes only after both Pruning calls).

    Returns (answer, iterations, distance_evaluations) where the distance
    count follows the per-iteration tally r1 + 3 r2 + 2 r1' of Section
    4.3.3 (r1, r2: sizes of s_i, s_j at the start of an iteration; r1': size
    of s_i after it has been pruned).
    """
    T = int(eps) ** 2
    si = [tuple(int(v) for v in p) for p in si]
    sj = [tuple(int(v) for v in p) for p in sj]
    alive_i = list(range(len(si)))
    alive_j = list(range(len(sj)))
    p = start
    iters = 0
    dist_evals = 0

    def nearest(src, idxs, pts):
        best, bd = None, None
        for k in idxs:
            dd = sqdist(src, pts[k])
            if bd is None or dd < bd:
                best, bd = k, dd
        return best, bd

    def pruning(s_a, alive_a, s_b, alive_b, pa, qb):
        # lambda = max over y in s_b of asin(eps/|pa y|) + angle(pa->qb, pa->y)
        P, Q = s_a[pa], s_b[qb]
        pq = [b - a for a, b in zip(P, Q)]
        npq = math.sqrt(sqdist(P, Q))
        lam = 0.0
        for k in alive_b:
            Y = s_b[k]
            py = [b - a for a, b in zip(P, Y)]
            npy = math.sqrt(sqdist(P, Y))
            c = sum(a * b for a, b in zip(pq, py)) / (npq * npy)
            lam_y = math.asin(min(1.0, eps / npy)) + math.acos(max(-1.0, min(1.0, c)))
            lam = max(lam, lam_y)
        dq = sqdist(P, Q)
        keep = []
        for k in alive_a:
            X = s_a[k]
            a = sqdist(X, P)
            # dist(x, p) < dist(p, q) - eps, exactly: sqrt(a) + eps < sqrt(dq)
            s = dq - T - a
            if s > 0 and 4 * T * a < s * s:
                continue
            px = [b - a_ for a_, b in zip(P, X)]
            npx = math.sqrt(a)
            c = sum(u * v for u, v in zip(pq, px)) / (npq * npx)
            theta = math.acos(max(-1.0, min(1.0, c)))
            if lam < math.pi and theta > lam + 1e-9:
                continue
            keep.append(k)
        return keep

    while True:
        iters += 1
        r1, r2 = len(alive_i), len(alive_j)
        q, dpq = nearest(si[p], alive_j, sj)
        if dpq <= T:
            dist_evals += r2
            return True, iters, dist_evals
        alive_i = pruning(si, alive_i, sj, alive_j, p, q)
        if not alive_i:
            dist_evals += r1 + 2 * r2
            return False, iters, dist_evals
        p, dqp = nearest(sj[q], alive_i, si)
        r1n = len(alive_i)
        if dqp <= T:
            dist_evals += r1 + 2 * r2 + r1n
            return True, iters, dist_evals
        alive_j = pruning(sj, alive_j, si, alive_i, q, p)
        dist_evals += r1 + 3 * r2 + 2 * r1n
        if not alive_j:
            return False, iters, dist_evals


# --------------------------------------------------------------------------
# Core grids and the merge graph (Section 3.2).
# --------------------------------------------------------------------------
def cell_assignment(points, eps: int):
    """(cells, counts, cell_of_point) with cells in lexicographic order."""
    ids = cell_ids(points, eps)
    cells, inverse, counts = np.unique(ids, axis=0, return_inverse=True, return_counts=True)
    return cells, counts, inverse.reshape(-1)
