"""Pins for the FP64 reference of the learned pair scorer."""
import numpy as np

from oracle import mlp


def _batch(seed, B=32):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((B, mlp.N_IN))
    t = np.stack([rng.integers(0, 2, B), rng.integers(0, 2, B), rng.integers(0, 2, B)], axis=1).astype(float)
    return x, t


def test_parameter_count():
    assert mlp.N_PARAMS == 16 * 64 + 64 + 64 * 64 + 64 + 2 * 64 + 2 == 5378


def test_gradient_matches_central_differences():
    theta = mlp.init(3)
    x, t = _batch(4)
    g = mlp.grad(theta, x, t)
    rng = np.random.default_rng(5)
    idx = rng.choice(mlp.N_PARAMS, size=120, replace=False)
    # biases of the last layers too
    idx = np.concatenate([idx, [mlp.N_PARAMS - 1, mlp.N_PARAMS - 2, 16 * 64 + 3]])
    num = mlp.numeric_grad(theta, x, t, idx)
    err = np.abs(num - g[idx]) / np.maximum(1e-8, np.abs(num) + np.abs(g[idx]))
    assert np.max(err[np.abs(num) > 1e-7]) < 1e-3


def test_forward_closed_form():
    # W1 = [I_16; 0], W2 = I, W3 row 0 sums h2, row 1 = 0, biases chosen by hand
    p = {name: np.zeros(shape) for name, shape in mlp.SHAPES}
    p["W1"][:16, :16] = np.eye(16)
    p["W2"] = np.eye(64)
    p["W3"][0, :] = 1.0
    p["b3"][:] = [0.5, -2.0]
    theta = mlp.pack(p)
    x = np.array([[1.0, -2.0, 3.0] + [0.0] * 13])
    z, _ = mlp.forward(theta, x)
    # relu keeps 1 and 3, drops -2
    assert np.allclose(z, [[4.5, -2.0]])
    # loss for y0 = 1, y1 = 0, w1 = 1: softplus(-4.5) + 0.5 softplus(-2)
    want = np.log1p(np.exp(-4.5)) + 0.5 * np.log1p(np.exp(-2.0))
    assert np.isclose(mlp.loss(theta, x, np.array([[1.0, 0.0, 1.0]])), want)


def test_adam_decreases_loss_on_separable_data():
    rng = np.random.default_rng(8)
    x = rng.standard_normal((256, 16))
    y = (x[:, 0] + 0.5 * x[:, 1] > 0).astype(float)
    t = np.stack([y, 1 - y, np.ones_like(y)], axis=1)
    theta = mlp.init(1)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss(theta, x, t)
    for s in range(1, 201):
        theta, m, v = mlp.adam_step(theta, m, v, mlp.grad(theta, x, t), s, lr=3e-3)
    assert mlp.loss(theta, x, t) < 0.3 * l0
