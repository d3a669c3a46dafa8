"""FP64 reference of the learned pair scorer.  TEST INFRASTRUCTURE ONLY.

The scorer is this project's own addition (the paper picks FastMerging's
start point at random and visits grid pairs in BFS or LDF order): a
16 -> 64 -> 64 -> 2 ReLU perceptron over features of an ordered pair of core
grids.  Output 0 is the logit that the pair merges; output 1 is the logit
that FastMerging costs fewer distance evaluations when it starts from the
second grid.  Neither output can change a merge decision: FastMerging
decides every pair exactly (Theorem 2), the scorer only orders the tests and
picks the starting side.

Parameter vector layout (5378 values, the layout of the FP16 blob):
W1 [64 x 16] row-major, b1 [64], W2 [64 x 64], b2 [64], W3 [2 x 64], b3 [2].

Loss of one sample with targets (y0, y1, w1):
    softplus(z0) - y0 z0  +  LAMBDA * w1 * (softplus(z1) - y1 z1)
(binary cross-entropy with logits), averaged over the batch.

Parity unpinned by the paper (this model is not in it); pinned here by
central finite differences, closed forms on hand-set weights, and closed
forms of the Adam recursion (first step, constant gradient, a single
gradient followed by zeros, scale invariance).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 16, 64, 2
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)  # 5378
LAMBDA = 0.5


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def init(seed: int = 0):
    """He-style initialisation (weights N(0, 2/fan_in), zero biases)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            p[name] = rng.standard_normal(shape) * np.sqrt(2.0 / shape[1])
        else:
            p[name] = np.zeros(shape)
    return pack(p)


def _to_half(a):
    """Round to the nearest IEEE binary16 value (ties to even), kept in FP64."""
    return np.asarray(a, dtype=np.float64).astype(np.float16).astype(np.float64)


def forward(theta, x, hidden_fp16=False):
    """Logits z [B, 2] and the hidden activations.

    hidden_fp16: round each hidden activation h = relu(a) to binary16 before
    the next layer uses it (the storage precision of the FP16 scorer, whose
    kernels keep hidden activations as halves); everything else stays FP64.
    The gradient then follows the rounded forward pass, with the rounding
    itself treated as the identity (straight-through), as the kernels do."""
    p = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    rnd = _to_half if hidden_fp16 else (lambda a: a)
    a1 = x @ p["W1"].T + p["b1"]
    h1 = rnd(np.maximum(a1, 0.0))
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = rnd(np.maximum(a2, 0.0))
    z = h2 @ p["W3"].T + p["b3"]
    return z, (x, a1, h1, a2, h2)


def softplus(z):
    return np.logaddexp(0.0, z)


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def loss(theta, x, t, hidden_fp16=False):
    """Mean loss over the batch; t [B, 3] = (y0, y1, w1)."""
    z, _ = forward(theta, x, hidden_fp16)
    t = np.asarray(t, dtype=np.float64)
    l0 = softplus(z[:, 0]) - t[:, 0] * z[:, 0]
    l1 = softplus(z[:, 1]) - t[:, 1] * z[:, 1]
    return float(np.mean(l0 + LAMBDA * t[:, 2] * l1))


def grad(theta, x, t, hidden_fp16=False):
    """Gradient of loss() by back-propagation (chain rule, layer by layer)."""
    p = unpack(theta)
    z, (x, a1, h1, a2, h2) = forward(theta, x, hidden_fp16)
    t = np.asarray(t, dtype=np.float64)
    B = x.shape[0]
    dz = np.empty_like(z)
    dz[:, 0] = (sigmoid(z[:, 0]) - t[:, 0]) / B
    dz[:, 1] = LAMBDA * t[:, 2] * (sigmoid(z[:, 1]) - t[:, 1]) / B
    g = {"W3": dz.T @ h2, "b3": dz.sum(axis=0)}
    dh2 = dz @ p["W3"]
    da2 = dh2 * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * (a1 > 0)
    g["W1"] = da1.T @ x
    g["b1"] = da1.sum(axis=0)
    return pack(g)


def numeric_grad(theta, x, t, idx, h=1e-6):
    """Central differences of loss() for the parameters in idx."""
    out = np.empty(len(idx))
    for k, i in enumerate(idx):
        tp = np.array(theta, dtype=np.float64)
        tm = tp.copy()
        tp[i] += h
        tm[i] -= h
        out[k] = (loss(tp, x, t) - loss(tm, x, t)) / (2 * h)
    return out


def block_slices():
    """Name and slice of each parameter block in the flat vector."""
    out, o = [], 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out.append((name, slice(o, o + k)))
        o += k
    return out


def adam_step(theta, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015, Algorithm 1), step counted from 1:
    first and second moment estimates, their bias corrections
    1 - b1^step and 1 - b2^step, and the step lr * m_hat / (sqrt(v_hat) + eps)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
