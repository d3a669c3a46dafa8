"""Training the learned proposal of the merge step.

The scorer (16 -> 64 -> 64 -> 2, see include/gritdbscan.h) learns from
merges the method itself performs: after a clustering, the library harvests
pairs of neighbouring core grids, runs FastMerging on each from both sides,
and records the answer and which side was cheaper.  Training runs on the GPU
in the library's own FP16 kernels (FP32 master weights, Adam).
"""
from __future__ import annotations

import os

import numpy as np

from . import MLP_PARAMS, Context

BLOB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "proposal_fp16.bin")

_SHAPES = [(64, 16), (64,), (64, 64), (64,), (2, 64), (2,)]


def init_params(seed: int = 0) -> np.ndarray:
    """He initialisation: weights N(0, 2 / fan_in), zero biases (float32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in _SHAPES:
        if len(shape) == 2:
            parts.append(rng.standard_normal(shape) * np.sqrt(2.0 / shape[1]))
        else:
            parts.append(np.zeros(shape))
    out = np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
    assert out.shape == (MLP_PARAMS,)
    return out


def harvest_from(ctx: Context, points, eps, minpts, target: int, seed: int = 0):
    """Cluster one workload and harvest about `target` pairs from it (with
    the neighbour lists of every grid written out, which harvesting reads)."""
    from . import GD_OPT_NEIGHBOR_MODE
    ctx.set_option(GD_OPT_NEIGHBOR_MODE, 1)
    try:
        ctx.dbscan(points, eps, minpts)
    finally:
        ctx.set_option(GD_OPT_NEIGHBOR_MODE, 0)
    st = ctx.stats()
    pairs = max(1, st["neighbor_entries"] // 2)
    keep_mod = max(1, pairs // max(target, 1))
    return ctx.harvest(cap=target, keep_mod=keep_mod, seed=seed)


def train(ctx: Context, X, T, steps: int = 3000, batch: int = 256, lr: float = 2e-3, seed: int = 0):
    """Train on harvested (X, T) device tensors.  Returns (fp16 blob as numpy,
    per-step losses as numpy)."""
    import torch
    dev = X.device
    S = X.shape[0]
    if S == 0:
        raise ValueError("no training samples")
    rng = np.random.default_rng(seed)
    order = np.concatenate([rng.permutation(S) for _ in range(-(-steps * batch // S))])[: steps * batch]
    order_d = torch.from_numpy(order.astype(np.int32)).to(dev)
    params = torch.from_numpy(init_params(seed)).to(dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    losses, blob = ctx.mlp_train(X, T, order_d, steps, batch, lr, params, m, v)
    torch.cuda.synchronize()
    return blob.cpu().numpy().astype(np.float16), losses.cpu().numpy()


def save_blob(blob: np.ndarray, path: str = BLOB_PATH):
    np.asarray(blob, dtype=np.float16).tofile(path)


def load_blob(path: str = BLOB_PATH) -> np.ndarray:
    b = np.fromfile(path, dtype=np.float16)
    if b.shape != (MLP_PARAMS,):
        raise ValueError(f"{path}: expected {MLP_PARAMS} FP16 values, found {b.shape}")
    return b
