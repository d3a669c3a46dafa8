"""CPU oracle for exact grid DBSCAN.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library and never
imports it.

* ``dbscan`` / ``dbscan_brute`` -- plain DBSCAN (Section 3.1, Definitions
  1-5) by pointwise eps range queries, in C (``dbscan_oracle.c``), with
  canonical labels: a cluster's id is the smallest index among its core
  points, a border point joins the cluster of its lowest-index core
  neighbour, noise is -1.
* ``neighbor_count_brute`` -- |N(p)| for sampled points by an O(n) scan.
* ``steps`` -- definitions of the intermediate results (cell identifiers of
  Eq. (1), neighbouring grids, MinDist of Definition 6, the merge graph)
  and the FP64 reference of the learned pair scorer.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dbscan_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-std=c11", "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        lib.oracle_dbscan.argtypes = [vp, i64, i32, i64, i64, vp, vp, i32]
        lib.oracle_dbscan.restype = ctypes.c_int
        lib.oracle_dbscan_brute.argtypes = [vp, i64, i32, i64, i64, vp, vp]
        lib.oracle_dbscan_brute.restype = ctypes.c_int
        lib.oracle_neighbor_count_brute.argtypes = [vp, i64, i32, i64, vp, i64, vp, i32]
        lib.oracle_neighbor_count_brute.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _prep(points, eps):
    x = np.ascontiguousarray(np.asarray(points))
    if x.ndim != 2:
        raise ValueError("points must be (n, d)")
    if not np.issubdtype(x.dtype, np.integer):
        xi = np.rint(x)
        if not np.array_equal(xi, x):
            raise ValueError("oracle needs integer-valued coordinates")
        x = xi
    x = np.ascontiguousarray(x.astype(np.int32))
    if int(eps) != eps or eps < 1:
        raise ValueError("oracle needs a positive integer eps")
    return x, int(eps)


def dbscan(points, eps, minpts, nthreads: int = 0):
    """(labels int32[n], core uint8[n]) by range queries over eps-side cells."""
    x, eps = _prep(points, eps)
    n, d = x.shape
    labels = np.empty(n, np.int32)
    core = np.empty(n, np.uint8)
    rc = _load().oracle_dbscan(x.ctypes.data, n, d, eps, int(minpts),
                               labels.ctypes.data, core.ctypes.data, int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_dbscan failed with status {rc}")
    return labels, core


def dbscan_brute(points, eps, minpts):
    """Same result by an O(n^2) scan of all pairs; tiny inputs only."""
    x, eps = _prep(points, eps)
    n, d = x.shape
    labels = np.empty(n, np.int32)
    core = np.empty(n, np.uint8)
    rc = _load().oracle_dbscan_brute(x.ctypes.data, n, d, eps, int(minpts),
                                     labels.ctypes.data, core.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"oracle_dbscan_brute failed with status {rc}")
    return labels, core


def neighbor_count_brute(points, eps, qidx, nthreads: int = 0):
    """|N(p)| (closed eps-ball, p included) for each p in ``qidx``."""
    x, eps = _prep(points, eps)
    n, d = x.shape
    q = np.ascontiguousarray(np.asarray(qidx, dtype=np.int64))
    out = np.empty(q.shape[0], np.int64)
    rc = _load().oracle_neighbor_count_brute(x.ctypes.data, n, d, eps, q.ctypes.data,
                                             q.shape[0], out.ctypes.data, int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_neighbor_count_brute failed with status {rc}")
    return out


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def core_components(points, core, radius):
    """Canonical component labels of the core points under the graph with an
    edge wherever two core points are within `radius` (exact integer squared
    distances): each core point gets the smallest index of its component,
    every other point -1.  With radius = eps this is DBSCAN's partition of
    the core points (Definitions 2-5); with eps + delta it is the coarsest
    partition the approximate merge of Section 4.3.3 (the remark on numerical
    error) may produce.  Pairs come from scipy's k-d tree (a library
    neighbour search, queried with a half-unit slack) and are kept only when
    their exact squared distance is at most radius^2."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    from scipy.spatial import cKDTree
    x, r = _prep(points, radius)
    core = np.asarray(core).astype(bool)
    idx = np.nonzero(core)[0]
    labels = np.full(x.shape[0], -1, np.int64)
    if idx.size == 0:
        return labels.astype(np.int32)
    pts = x[idx].astype(np.int64)
    pairs = cKDTree(pts).query_pairs(r + 0.5, output_type="ndarray")
    if pairs.size:
        d2 = ((pts[pairs[:, 0]] - pts[pairs[:, 1]]) ** 2).sum(axis=1)
        pairs = pairs[d2 <= r * r]
    m = idx.size
    g = coo_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])), shape=(m, m)) if len(pairs) else \
        coo_matrix((m, m))
    _, comp = connected_components(g, directed=False)
    first = np.full(comp.max() + 1, np.iinfo(np.int64).max)
    np.minimum.at(first, comp, idx)
    labels[idx] = first[comp]
    return labels.astype(np.int32)
