"""Exact grid DBSCAN (GriT-DBSCAN) on AMD MI355X: Python binding.

Thin ctypes layer over ``libgritdbscan.so`` (declared in
``include/gritdbscan.h``).  It only marshals arguments: torch supplies the
device memory and the stream; every step of the clustering runs in the
library's HIP kernels.  There is no CPU fallback: without the built library
every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GRITDBSCAN_LIBRARY selects another build of the same library (for example
# the host-sanitizer variant of build.py); the default is the in-tree one
LIB_PATH = os.environ.get("GRITDBSCAN_LIBRARY") or os.path.join(_HERE, "libgritdbscan.so")

GD_OK, GD_EINVAL, GD_ERANGE, GD_ENOMEM, GD_EDEVICE, GD_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
GD_OPT_STATS, GD_OPT_LDF_ORDER, GD_OPT_WORKSPACE_LIMIT, GD_OPT_TIMING, GD_OPT_GRAPH = 1, 2, 3, 4, 5
GD_OPT_TILE_POINTS, GD_OPT_MERGE_WAVES, GD_OPT_NEIGHBOR_MODE, GD_OPT_MERGE_ORDER = 6, 7, 8, 9
GD_OPT_APPROX_DELTA, GD_OPT_NEIGHBOR_QUERY, GD_OPT_GRID_LANES, GD_OPT_PACKED_ROWS = 10, 11, 12, 13
NOALLOC_SCRATCH_BYTES = 256 << 20
PHASE_COUNT = 14
EPS_MAX = 21845  # largest eps of the 32-bit distance path (GD_EPS_MAX); larger eps use 64 bits
D_MAX = 8


class GDError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_status_name(status)}: {message}")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in ("n",)] + [
        ("d", ctypes.c_int32), ("key_bits", ctypes.c_int32)] + [
        (name, ctypes.c_int64) for name in (
            "grids", "neighbor_entries", "core_points", "core_grids", "dense_grids",
            "max_grid_points", "merge_pairs", "merge_skipped", "merge_tests", "merge_yes",
            "merge_iterations", "merge_max_iterations", "merge_distances", "core_distances",
            "border_points", "noise_points", "clusters", "merge_set_points", "graph_replays",
            "core_candidates", "core_neighbor_grids", "neighbor_walk")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Tuning(ctypes.Structure):
    _fields_ = [("tile_points", ctypes.c_int32), ("merge_waves", ctypes.c_int32), ("grid_lanes", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class Instance(ctypes.Structure):
    _fields_ = [("points", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("minpts", ctypes.c_int32), ("eps", ctypes.c_double), ("labels", ctypes.c_void_p),
                ("core_flags", ctypes.c_void_p)]


_lib = None

EXPORTS = ("gd_create", "gd_destroy", "dbscan", "dbscan_noalloc", "dbscan_batched", "gd_set_option", "gd_get_stats",
           "gd_debug_grids", "gd_debug_neighbors", "gd_debug_core", "gd_merge_test",
           "gd_get_phase_times", "gd_phase_name", "gd_set_proposal", "gd_proposal_harvest",
           "gd_mlp_train", "gd_mlp_grad", "gd_mlp_forward", "gd_last_error", "gd_status_string", "gd_autotune",
           "gd_set_tuning_file")
MLP_PARAMS = 5378
MLP_FEATURES = 16


def load_library(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2210_07580_amd/build.py "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.gd_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
    lib.gd_create.restype = ctypes.c_int
    lib.gd_destroy.argtypes = [vp]
    lib.gd_destroy.restype = None
    lib.dbscan.argtypes = [vp, vp, i64, i32, dbl, i32, vp, vp, vp]
    lib.dbscan.restype = ctypes.c_int
    lib.dbscan_noalloc.argtypes = [vp, vp, i64, i32, dbl, i32, vp, vp, vp]
    lib.dbscan_noalloc.restype = ctypes.c_int
    lib.dbscan_batched.argtypes = [vp, ctypes.POINTER(Instance), i32, vp]
    lib.dbscan_batched.restype = ctypes.c_int
    lib.gd_set_option.argtypes = [vp, ctypes.c_int, i64]
    lib.gd_set_option.restype = ctypes.c_int
    lib.gd_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    lib.gd_get_stats.restype = ctypes.c_int
    lib.gd_debug_grids.argtypes = [vp, ctypes.POINTER(i64), vp, vp, vp]
    lib.gd_debug_grids.restype = ctypes.c_int
    lib.gd_debug_neighbors.argtypes = [vp, vp, vp]
    lib.gd_debug_neighbors.restype = ctypes.c_int
    lib.gd_debug_core.argtypes = [vp, vp, vp]
    lib.gd_debug_core.restype = ctypes.c_int
    lib.gd_merge_test.argtypes = [vp, vp, i64, i32, dbl, vp, i64, vp, vp, vp]
    lib.gd_merge_test.restype = ctypes.c_int
    lib.gd_get_phase_times.argtypes = [vp, vp, i32]
    lib.gd_get_phase_times.restype = ctypes.c_int
    lib.gd_phase_name.argtypes = [i32]
    lib.gd_phase_name.restype = ctypes.c_char_p
    lib.gd_set_proposal.argtypes = [vp, vp]
    lib.gd_set_proposal.restype = ctypes.c_int
    lib.gd_proposal_harvest.argtypes = [vp, ctypes.c_uint32, ctypes.c_uint32, i64, vp, vp, vp,
                                        ctypes.POINTER(i64), vp]
    lib.gd_proposal_harvest.restype = ctypes.c_int
    lib.gd_mlp_train.argtypes = [vp, vp, vp, i64, vp, i32, i32, ctypes.c_float, i32, vp, vp, vp, vp, vp, vp]
    lib.gd_mlp_train.restype = ctypes.c_int
    lib.gd_mlp_grad.argtypes = [vp, vp, vp, vp, i32, vp, vp, vp, vp]
    lib.gd_mlp_grad.restype = ctypes.c_int
    lib.gd_mlp_forward.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.gd_mlp_forward.restype = ctypes.c_int
    lib.gd_autotune.argtypes = [vp, ctypes.POINTER(Instance), i32, vp, ctypes.POINTER(Tuning), i32,
                                ctypes.POINTER(i32)]
    lib.gd_autotune.restype = ctypes.c_int
    lib.gd_set_tuning_file.argtypes = [vp, ctypes.c_char_p]
    lib.gd_set_tuning_file.restype = ctypes.c_int
    lib.gd_last_error.argtypes = [vp]
    lib.gd_last_error.restype = ctypes.c_char_p
    lib.gd_status_string.argtypes = [ctypes.c_int]
    lib.gd_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _status_name(status: int) -> str:
    names = {0: "GD_OK", -1: "GD_EINVAL", -2: "GD_ERANGE", -3: "GD_ENOMEM",
             -4: "GD_EDEVICE", -5: "GD_EUNSUPPORTED"}
    return names.get(status, f"status {status}")


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream_handle(stream) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


class Context:
    """One library context (device workspace, options, last-call stats)."""

    def __init__(self, device: int = 0):
        lib = load_library()
        h = ctypes.c_void_p()
        rc = lib.gd_create(ctypes.byref(h), int(device))
        if rc != GD_OK:
            raise GDError(rc, f"gd_create(device={device}) failed")
        self._h = h
        self.device = int(device)

    def close(self):
        if getattr(self, "_h", None):
            load_library().gd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int):
        if rc != GD_OK:
            msg = load_library().gd_last_error(self._h).decode()
            raise GDError(rc, msg)

    def set_option(self, option: int, value: int):
        self._check(load_library().gd_set_option(self._h, int(option), int(value)))

    def dbscan(self, points, eps, minpts: int, labels=None, core_flags=None, stream=None):
        """Cluster ``points`` (torch float32 [n, d] on the context's device).

        Returns (labels int32 [n], core_flags uint8 [n]) as device tensors.
        """
        return self._single(load_library().dbscan, points, eps, minpts, labels, core_flags, stream)

    def dbscan_noalloc(self, points, eps, minpts: int, labels, core_flags, stream=None):
        """dbscan() into caller-given output tensors, with every workspace
        buffer taken from the library's fixed per-device scratch array (the
        call allocates nothing)."""
        if labels is None or core_flags is None:
            raise ValueError("dbscan_noalloc writes into given labels and core_flags tensors")
        return self._single(load_library().dbscan_noalloc, points, eps, minpts, labels, core_flags, stream)

    def _single(self, fn, points, eps, minpts, labels, core_flags, stream):
        import torch
        if not isinstance(points, torch.Tensor) or points.dim() != 2:
            raise ValueError("points must be a 2-D torch tensor")
        if points.device.type != "cuda":
            raise ValueError("points must live on the GPU")
        if points.dtype != torch.float32:
            raise ValueError("points must be float32")
        pts = points.contiguous()
        n, d = pts.shape
        if labels is None:
            labels = torch.empty(n, dtype=torch.int32, device=pts.device)
        if core_flags is None:
            core_flags = torch.empty(n, dtype=torch.uint8, device=pts.device)
        if labels.numel() != n or core_flags.numel() != n or labels.dtype != torch.int32 \
                or core_flags.dtype != torch.uint8:
            raise ValueError("labels must be int32 [n] and core_flags uint8 [n]")
        rc = fn(self._h, _ptr(pts), int(n), int(d), float(eps), int(minpts), _ptr(labels), _ptr(core_flags),
                _stream_handle(stream))
        self._check(rc)
        return labels, core_flags

    def _descriptors(self, problems, outs=None):
        import torch
        descs = (Instance * max(len(problems), 1))()
        given, res, keep = outs, [], []
        for k, (pts, eps, minpts) in enumerate(problems):
            if pts.dtype != torch.float32 or pts.dim() != 2 or pts.device.type != "cuda":
                raise ValueError(f"instance {k}: points must be a float32 [n, d] GPU tensor")
            pts = pts.contiguous()
            n, d = pts.shape
            if given is not None:
                lab, core = given[k]
                if lab.numel() != n or core.numel() != n or lab.dtype != torch.int32 or core.dtype != torch.uint8:
                    raise ValueError(f"instance {k}: output tensors must be int32 [n] and uint8 [n]")
            else:
                lab = torch.empty(n, dtype=torch.int32, device=pts.device)
                core = torch.empty(n, dtype=torch.uint8, device=pts.device)
            descs[k] = Instance(_ptr(pts) if n else None, int(n), int(d), int(minpts), float(eps),
                                _ptr(lab) if n else None, _ptr(core) if n else None)
            keep.append(pts)
            res.append((lab, core))
        return descs, res, keep

    def autotune(self, problems, stream=None):
        """Time the batch under every tunable configuration and keep the
        fastest (or apply the tuning file's entry for this batch shape).
        Returns (chosen {tile_points, merge_waves, grid_lanes} or None when
        the file supplied it, all timings)."""
        descs, _, keep = self._descriptors(problems)
        res = (Tuning * 64)()
        cnt = ctypes.c_int32()
        self._check(load_library().gd_autotune(self._h, descs, len(problems), _stream_handle(stream), res, 64,
                                               ctypes.byref(cnt)))
        rows = [{"tile_points": r.tile_points, "merge_waves": r.merge_waves, "grid_lanes": r.grid_lanes, "ms": r.ms}
                for r in res[:cnt.value]]
        best = min(rows, key=lambda r: r["ms"]) if rows else None
        return ({k: best[k] for k in ("tile_points", "merge_waves", "grid_lanes")} if best else None), rows

    def set_tuning_file(self, path):
        """JSON file of tuned configurations by batch shape (None: off)."""
        self._check(load_library().gd_set_tuning_file(self._h, None if path is None else os.fsencode(path)))

    def dbscan_batched(self, problems, stream=None, outs=None):
        """Cluster many instances in one pass.  ``problems``: list of
        (points float32 [n_k, d_k] on the device, eps_k, minpts_k).  Returns
        a list of (labels, core_flags) device tensors, one per instance
        (``outs``, when given, is such a list to write into)."""
        descs, outs, keep = self._descriptors(problems, outs)
        rc = load_library().dbscan_batched(self._h, descs, len(problems), _stream_handle(stream))
        self._check(rc)
        return outs

    def set_proposal(self, fp16_params):
        """Use the learned proposal (numpy float16 [5378]); None switches it off."""
        lib = load_library()
        if fp16_params is None:
            self._check(lib.gd_set_proposal(self._h, None))
            return
        blob = np.ascontiguousarray(np.asarray(fp16_params, dtype=np.float16))
        if blob.shape != (MLP_PARAMS,):
            raise ValueError(f"proposal needs {MLP_PARAMS} FP16 values")
        self._check(lib.gd_set_proposal(self._h, blob.ctypes.data))

    def harvest(self, cap: int, keep_mod: int = 1, seed: int = 0, stream=None):
        """Training pairs from the last dbscan() call: (features fp16 [k,16],
        targets f32 [k,3], costs f32 [k,3]) device tensors."""
        import torch
        dev = torch.device("cuda", self.device)
        X = torch.empty((max(cap, 1), MLP_FEATURES), dtype=torch.float16, device=dev)
        T = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=dev)
        C = torch.empty((max(cap, 1), 3), dtype=torch.float32, device=dev)
        cnt = ctypes.c_int64()
        rc = load_library().gd_proposal_harvest(self._h, int(seed), int(keep_mod), int(cap), _ptr(X), _ptr(T),
                                                _ptr(C), ctypes.byref(cnt), _stream_handle(stream))
        self._check(rc)
        k = cnt.value
        return X[:k], T[:k], C[:k]

    def mlp_train(self, X, T, order, steps: int, batch: int, lr: float, params, adam_m, adam_v,
                  adam_t0: int = 0, stream=None):
        """Adam steps on the GPU; returns (losses f32 [steps], blob fp16 [5378])."""
        import torch
        loss = torch.empty(max(steps, 1), dtype=torch.float32, device=params.device)
        blob = torch.empty(MLP_PARAMS, dtype=torch.float16, device=params.device)
        rc = load_library().gd_mlp_train(self._h, _ptr(X), _ptr(T), int(X.shape[0]), _ptr(order), int(steps),
                                         int(batch), float(lr), int(adam_t0), _ptr(params), _ptr(adam_m),
                                         _ptr(adam_v), _ptr(loss), _ptr(blob), _stream_handle(stream))
        self._check(rc)
        return loss[:steps], blob

    def mlp_grad(self, X, T, order, batch: int, params, stream=None):
        """(gradient f32 [5378], mean loss) of one batch, no update."""
        import torch
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=params.device)
        loss = torch.empty(1, dtype=torch.float32, device=params.device)
        rc = load_library().gd_mlp_grad(self._h, _ptr(X), _ptr(T), _ptr(order), int(batch), _ptr(params),
                                        _ptr(g), _ptr(loss), _stream_handle(stream))
        self._check(rc)
        return g, float(loss.item())

    def mlp_forward(self, X, blob, stream=None):
        import torch
        Z = torch.empty((X.shape[0], 2), dtype=torch.float32, device=X.device)
        rc = load_library().gd_mlp_forward(self._h, _ptr(X), int(X.shape[0]), _ptr(blob), _ptr(Z),
                                           _stream_handle(stream))
        self._check(rc)
        return Z

    def stats(self) -> dict:
        s = Stats()
        self._check(load_library().gd_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def phase_times(self) -> dict:
        """GPU milliseconds per phase of the last call made with GD_OPT_TIMING on."""
        lib = load_library()
        ms = np.zeros(PHASE_COUNT, np.float64)
        self._check(lib.gd_get_phase_times(self._h, ms.ctypes.data, PHASE_COUNT))
        return {lib.gd_phase_name(i).decode(): float(ms[i]) for i in range(PHASE_COUNT)}

    def debug_grids(self):
        """(sorted_index[n], grid_start[|Gs|+1], grid_ids[|Gs|, d]) of the last call."""
        lib = load_library()
        ng = ctypes.c_int64()
        self._check(lib.gd_debug_grids(self._h, ctypes.byref(ng), None, None, None))
        st = self.stats()
        n, d = st["n"], st["d"]
        sidx = np.empty(n, np.uint32)
        gs = np.empty(ng.value + 1, np.uint32)
        ids = np.empty((ng.value, d), np.int32)
        self._check(lib.gd_debug_grids(self._h, ctypes.byref(ng), sidx.ctypes.data,
                                       gs.ctypes.data, ids.ctypes.data))
        return sidx, gs, ids

    def debug_neighbors(self):
        """(offsets[|Gs|+1] uint64, neighbors[total] uint32) of the last call."""
        lib = load_library()
        st = self.stats()
        off = np.empty(st["grids"] + 1, np.uint64)
        nei = np.empty(max(st["neighbor_entries"], 1), np.uint32)
        self._check(lib.gd_debug_neighbors(self._h, off.ctypes.data, nei.ctypes.data))
        return off, nei[: st["neighbor_entries"]]

    def debug_core(self):
        """(core_flags in sorted order [n], grid_label [|Gs|]) of the last call."""
        lib = load_library()
        st = self.stats()
        core = np.empty(st["n"], np.uint8)
        lab = np.empty(st["grids"], np.int32)
        self._check(lib.gd_debug_core(self._h, core.ctypes.data, lab.ctypes.data))
        return core, lab

    def merge_test(self, points_soa, pairs, eps, with_iterations: bool = False, stream=None):
        """FastMerging on pairs of point runs.  ``points_soa``: torch int32
        [d, m] on the device; ``pairs``: torch int32/uint32 [npairs, 4]
        (a_begin, a_count, b_begin, b_count).  Returns uint8 answers (and
        iteration counts)."""
        import torch
        d, m = points_soa.shape
        pts = points_soa.contiguous().to(torch.int32)
        pr = pairs.contiguous().to(torch.int32)
        npairs = pr.shape[0]
        ans = torch.empty(npairs, dtype=torch.uint8, device=pts.device)
        its = torch.empty(npairs, dtype=torch.int32, device=pts.device) if with_iterations else None
        rc = load_library().gd_merge_test(self._h, _ptr(pts), int(m), int(d), float(eps), _ptr(pr),
                                          int(npairs), _ptr(ans), _ptr(its), _stream_handle(stream))
        self._check(rc)
        return (ans, its) if with_iterations else ans


_default_ctx = {}


def dbscan(points, eps, minpts: int, stream=None):
    """Exact DBSCAN of ``points`` (torch float32 [n, d] on a GPU, integer
    valued).  Returns (labels int32, core_flags uint8) on the same device:
    labels are the smallest input index of each cluster's core points, -1 for
    noise; border points join their lowest-index core neighbour's cluster."""
    dev = points.device.index or 0
    ctx = _default_ctx.get(dev)
    if ctx is None:
        ctx = _default_ctx[dev] = Context(dev)
    return ctx.dbscan(points, eps, minpts, stream=stream)
