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


def test_hidden_fp16_rounding_is_applied_and_gradient_matches_differences():
    theta = mlp.init(6)
    x, t = _batch(7, B=16)
    z64, (_, _, h1, _, _) = mlp.forward(theta, x)
    z16, (_, a1r, g1, a2r, g2) = mlp.forward(theta, x, hidden_fp16=True)
    # every hidden activation is a binary16 value, within half an ulp of the exact one
    assert np.array_equal(g1, g1.astype(np.float16).astype(np.float64))
    assert np.all(np.abs(g1 - h1) <= 2.0 ** -11 * np.abs(h1) + 2.0 ** -25)
    assert not np.array_equal(z16, z64)
    # the rounded forward pass's gradient, rounding taken as the identity: the
    # exact gradient of a network whose hidden layers carry fixed offsets
    # (h16 - h), so finite differences with those offsets frozen agree
    g = mlp.grad(theta, x, t, hidden_fp16=True)
    off1 = g1 - np.maximum(a1r, 0.0)
    off2 = g2 - np.maximum(a2r, 0.0)

    def frozen_loss(th):
        q = mlp.unpack(th)
        a1 = x @ q["W1"].T + q["b1"]
        k1 = np.maximum(a1, 0.0) + off1
        a2 = k1 @ q["W2"].T + q["b2"]
        k2 = np.maximum(a2, 0.0) + off2
        z = k2 @ q["W3"].T + q["b3"]
        l0 = mlp.softplus(z[:, 0]) - t[:, 0] * z[:, 0]
        l1 = mlp.softplus(z[:, 1]) - t[:, 1] * z[:, 1]
        return float(np.mean(l0 + mlp.LAMBDA * t[:, 2] * l1))

    assert np.isclose(frozen_loss(theta), mlp.loss(theta, x, t, hidden_fp16=True), rtol=0, atol=1e-12)
    idx = np.random.default_rng(2).choice(mlp.N_PARAMS, 80, replace=False)
    h = 1e-6
    num = []
    for i in idx:
        tp = np.array(theta)
        tm = tp.copy()
        tp[i] += h
        tm[i] -= h
        num.append((frozen_loss(tp) - frozen_loss(tm)) / (2 * h))
    num = np.array(num)
    err = np.abs(num - g[idx]) / np.maximum(1e-8, np.abs(num) + np.abs(g[idx]))
    assert np.max(err[np.abs(num) > 1e-7]) < 1e-3


def test_block_slices_cover_the_vector():
    sl = mlp.block_slices()
    assert [n for n, _ in sl] == ["W1", "b1", "W2", "b2", "W3", "b3"]
    assert sl[0][1].start == 0 and sl[-1][1].stop == mlp.N_PARAMS
    assert all(a[1].stop == b[1].start for a, b in zip(sl, sl[1:]))


def test_adam_first_step_is_a_normalised_gradient_step():
    # m0 = v0 = 0: after bias correction m_hat = g and v_hat = g^2, so every
    # parameter moves by -lr g / (|g| + eps): about -lr sign(g)
    rng = np.random.default_rng(11)
    theta = rng.standard_normal(500)
    g = rng.standard_normal(500) * np.logspace(-3, 2, 500)
    lr, eps = 0.01, 1e-8
    new, m, v = mlp.adam_step(theta, np.zeros(500), np.zeros(500), g, 1, lr=lr, eps=eps)
    assert np.allclose(new, theta - lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g, rtol=1e-12) and np.allclose(v, 0.001 * g * g, rtol=1e-12)


def test_adam_constant_gradient_closed_form():
    # g constant: m_k = (1 - b1^k) g and v_k = (1 - b2^k) g^2, so the bias
    # corrections make m_hat = g and v_hat = g^2 at every step and theta moves
    # by the same -lr g / (|g| + eps) each step
    rng = np.random.default_rng(12)
    theta0 = rng.standard_normal(64)
    g = rng.standard_normal(64)
    lr, eps, b1, b2 = 3e-3, 1e-8, 0.9, 0.999
    theta, m, v = theta0.copy(), np.zeros(64), np.zeros(64)
    for k in range(1, 41):
        theta, m, v = mlp.adam_step(theta, m, v, g, k, lr=lr)
        assert np.allclose(m, (1 - b1 ** k) * g, rtol=1e-12, atol=1e-15)
        assert np.allclose(v, (1 - b2 ** k) * g * g, rtol=1e-12, atol=1e-18)
    assert np.allclose(theta, theta0 - 40 * lr * g / (np.abs(g) + eps), rtol=1e-10, atol=1e-12)


def test_adam_moments_decay_by_their_own_beta():
    # one gradient g, then zeros: m_k = (1 - b1) b1^(k-1) g and
    # v_k = (1 - b2) b2^(k-1) g^2 (swapped betas or a wrong power fail here);
    # the step at k is lr (m_k / (1 - b1^k)) / (sqrt(v_k / (1 - b2^k)) + eps)
    g = np.array([2.0, -0.5, 1e-3])
    lr, eps, b1, b2 = 1e-2, 1e-8, 0.9, 0.999
    theta, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for k in range(1, 9):
        prev = theta
        theta, m, v = mlp.adam_step(theta, m, v, g if k == 1 else np.zeros(3), k, lr=lr)
        mk = (1 - b1) * b1 ** (k - 1) * g
        vk = (1 - b2) * b2 ** (k - 1) * g * g
        assert np.allclose(m, mk, rtol=1e-12) and np.allclose(v, vk, rtol=1e-12)
        want = lr * (mk / (1 - b1 ** k)) / (np.sqrt(vk / (1 - b2 ** k)) + eps)
        assert np.allclose(prev - theta, want, rtol=1e-10)


def test_adam_is_invariant_to_gradient_scale():
    # the update depends on g / sqrt(v): scaling every gradient by c > 0
    # leaves it unchanged (up to eps)
    rng = np.random.default_rng(13)
    gs = rng.standard_normal((6, 50))
    a = b = np.zeros(50)
    ma = va = mb = vb = np.zeros(50)
    for k, g in enumerate(gs, 1):
        a, ma, va = mlp.adam_step(a, ma, va, g, k, eps=0.0)
        b, mb, vb = mlp.adam_step(b, mb, vb, 1000.0 * g, k, eps=0.0)
    assert np.allclose(a, b, rtol=1e-10, atol=1e-14)
