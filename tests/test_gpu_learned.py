"""The learned proposal: FP16 kernels against the FP64 reference, training,
harvesting, and exactness (labels identical with and without a proposal)."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import mlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = G.Context(0)
    yield c
    c.close()


def _fp16(a):
    return np.asarray(a, dtype=np.float16)


def test_forward_matches_fp64(ctx):
    rng = np.random.default_rng(1)
    theta = _fp16(mlp.init(2))
    X = _fp16(rng.standard_normal((700, 16)))
    Z = ctx.mlp_forward(torch.from_numpy(X).cuda(), torch.from_numpy(theta).cuda()).cpu().numpy()
    want, _ = mlp.forward(theta.astype(np.float64), X.astype(np.float64))
    assert np.all(np.abs(Z - want) <= 2e-2 * (1 + np.abs(want)))


def _grad_case(seed, B=256):
    rng = np.random.default_rng(seed)
    theta32 = mlp.init(seed + 1).astype(np.float32)
    X = _fp16(rng.standard_normal((B, 16)))
    T = np.stack([rng.integers(0, 2, B), rng.integers(0, 2, B), rng.integers(0, 2, B)], 1).astype(np.float32)
    return theta32, X, T


def _gpu_grad(ctx, theta32, X, T):
    order = np.arange(len(X), dtype=np.int32)
    g, loss = ctx.mlp_grad(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), torch.from_numpy(order).cuda(),
                           len(X), torch.from_numpy(theta32).cuda())
    return g.cpu().numpy().astype(np.float64), loss


@pytest.mark.parametrize("seed", [3, 17])
def test_gradient_matches_fp64_per_block(ctx, seed):
    """Each parameter block of the kernel's gradient, element by element,
    against the FP64 reference run with the kernel's declared rounding (FP16
    weights, inputs and hidden activations).  What is left is FP32
    accumulation (relative 1e-6 per term) and the rare hidden activation
    whose FP32 pre-activation rounds to the neighbouring half (one FP16 ulp,
    2^-11 relative, in the terms that use it): per element at most
    |g - want| <= 1e-3 |want| + 1e-3 max|block|."""
    theta32, X, T = _grad_case(seed)
    g, loss = _gpu_grad(ctx, theta32, X, T)
    th16 = theta32.astype(np.float16).astype(np.float64)  # the kernel computes with FP16-rounded weights
    x64 = X.astype(np.float64)
    want = mlp.grad(th16, x64, T, hidden_fp16=True)
    for name, sl in mlp.block_slices():
        a, b = g[sl], want[sl]
        scale = np.max(np.abs(b))
        assert scale > 0, f"{name}: no gradient"
        bad = np.abs(a - b) > 1e-3 * np.abs(b) + 1e-3 * scale
        assert not bad.any(), f"{name}: {int(bad.sum())} of {b.size} elements off, worst {np.max(np.abs(a - b)) / scale:.2e}"
        assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b), name
    assert abs(loss - mlp.loss(th16, x64, T, hidden_fp16=True)) < 1e-4
    # and the plain FP64 network (no rounding) is within FP16 tolerance
    full = mlp.grad(th16, x64, T)
    assert np.linalg.norm(g - full) <= 3e-2 * np.linalg.norm(full)


@pytest.mark.parametrize("t0", [0, 5])
def test_adam_step_matches_reference(ctx, t0):
    """One gd_mlp_train step against oracle.mlp.adam_step fed the kernel's
    own gradient of the same batch, element by element: moments to FP32
    rounding, parameters to FP32 rounding of theta - lr m_hat / (sqrt(v_hat) + eps)."""
    theta32, X, T = _grad_case(23 + t0)
    rng = np.random.default_rng(99 + t0)
    B = len(X)
    if t0:
        m0 = (rng.standard_normal(mlp.N_PARAMS) * 1e-2).astype(np.float32)
        v0 = (rng.random(mlp.N_PARAMS) * 1e-4 + 1e-6).astype(np.float32)
    else:
        m0 = np.zeros(mlp.N_PARAMS, np.float32)
        v0 = np.zeros(mlp.N_PARAMS, np.float32)
    g, _ = _gpu_grad(ctx, theta32, X, T)
    lr = 2e-3
    P = torch.from_numpy(theta32.copy()).cuda()
    M = torch.from_numpy(m0.copy()).cuda()
    V = torch.from_numpy(v0.copy()).cuda()
    order = torch.arange(B, dtype=torch.int32, device="cuda")
    ctx.mlp_train(torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda(), order, 1, B, lr, P, M, V, adam_t0=t0)
    want_p, want_m, want_v = mlp.adam_step(theta32.astype(np.float64), m0.astype(np.float64),
                                           v0.astype(np.float64), g, t0 + 1, lr=lr)
    gm, gv, gp = (a.cpu().numpy().astype(np.float64) for a in (M, V, P))
    # FP32 error bounds (unit roundoff u = 2^-24, a few operations each): a
    # sum is off by at most ~u times the sum of its terms' magnitudes, which
    # matters where 0.9 m0 and 0.1 g cancel; the step inherits m's error
    u = 2.0 ** -24
    tol_m = 8 * u * (0.9 * np.abs(m0) + 0.1 * np.abs(g))
    assert np.all(np.abs(gm - want_m) <= tol_m + 1e-30)
    assert np.all(np.abs(gv - want_v) <= 8 * u * (0.999 * v0 + 0.001 * g * g) + 1e-30)
    c1, c2 = 1 - 0.9 ** (t0 + 1), 1 - 0.999 ** (t0 + 1)
    step = np.abs(theta32 - want_p)
    tol_step = lr * (tol_m / c1) / (np.sqrt(want_v / c2) + 1e-8) + 16 * u * step
    assert np.all(np.abs(gp - want_p) <= tol_step + 4 * u * np.abs(want_p) + 1e-30)
    if t0 == 0:  # the first step moves each parameter by lr g / (|g| + eps)
        assert np.allclose(theta32 - want_p, lr * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-12)


def test_training_reduces_loss(ctx):
    from paper_2210_07580_amd import proposal as P
    rng = np.random.default_rng(9)
    X = rng.standard_normal((4096, 16))
    y = (X[:, 0] - 0.7 * X[:, 3] > 0).astype(np.float32)
    s = (X[:, 1] > 0).astype(np.float32)
    T = np.stack([y, s, np.ones_like(y)], 1).astype(np.float32)
    blob, losses = P.train(ctx, torch.from_numpy(_fp16(X)).cuda(), torch.from_numpy(T).cuda(), steps=600,
                           batch=128, lr=3e-3)
    assert losses[-50:].mean() < 0.35 * losses[:20].mean()
    Z = ctx.mlp_forward(torch.from_numpy(_fp16(X)).cuda(), torch.from_numpy(blob).cuda()).cpu().numpy()
    assert ((Z[:, 0] > 0) == (y > 0.5)).mean() > 0.95


def test_harvest_targets_are_consistent(ctx):
    w = W.WORKLOADS["cfg1"].with_n(200_000)
    x = W.make_points(w)
    ctx.dbscan(torch.from_numpy(x.astype(np.float32)).cuda(), w.eps, w.minpts)
    X, T, C = ctx.harvest(cap=4000, keep_mod=3, seed=1)
    X, T, C = X.cpu().numpy(), T.cpu().numpy(), C.cpu().numpy()
    assert 100 < len(X) <= 4000
    assert np.isfinite(X.astype(np.float32)).all()
    assert set(np.unique(T)) <= {0.0, 1.0}
    assert (C >= 1).all()
    assert np.array_equal(T[:, 1] > 0.5, C[:, 2] < C[:, 1])
    assert np.array_equal(T[:, 2] > 0.5, C[:, 2] != C[:, 1])
    assert 0.0 < T[:, 0].mean() <= 1.0


def _random_blob(seed):
    return _fp16(mlp.init(seed))


@pytest.mark.parametrize("name,n", [("H", 150_000), ("cfg4", 200_000), ("cfg1", 150_000), ("cfg0", 10_000)])
def test_proposal_keeps_exact_labels(ctx, name, n):
    from paper_2210_07580_amd import proposal as P
    w = W.WORKLOADS[name].with_n(n)
    x = W.make_points(w)
    want = oracle.dbscan(x, w.eps, w.minpts)
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    blobs = [_random_blob(5)]
    if os.path.exists(P.BLOB_PATH):
        blobs.append(P.load_blob())
    try:
        for blob in blobs:
            ctx.set_proposal(blob)
            lab, core = ctx.dbscan(t, w.eps, w.minpts)
            assert np.array_equal(core.cpu().numpy(), want[1])
            assert np.array_equal(lab.cpu().numpy(), want[0])
    finally:
        ctx.set_proposal(None)


def test_trained_proposal_gain(ctx):
    """What the trained scorer buys over the plain method on the dense
    seed-spreader workload (300 points per step), at identical labels."""
    import paper_2210_07580_amd as G
    from paper_2210_07580_amd import proposal as P
    if not os.path.exists(P.BLOB_PATH):
        pytest.skip("no trained proposal committed")
    w = W.WORKLOADS["cfg4"].with_n(2_000_000)
    x = W.make_points(w)
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    ctx.set_option(G.GD_OPT_STATS, 1)
    try:
        l0, c0 = ctx.dbscan(t, w.eps, w.minpts)
        s0 = ctx.stats()
        ctx.set_proposal(P.load_blob())
        l1, c1 = ctx.dbscan(t, w.eps, w.minpts)
        s1 = ctx.stats()
    finally:
        ctx.set_proposal(None)
        ctx.set_option(G.GD_OPT_STATS, 0)
    assert torch.equal(l0, l1) and torch.equal(c0, c1)
    print(f"plain: tests {s0['merge_tests']} distances {s0['merge_distances']}; "
          f"learned: tests {s1['merge_tests']} distances {s1['merge_distances']}", flush=True)
    assert s1["merge_distances"] < s0["merge_distances"]


def test_trained_proposal_gain_on_large_core_sets(ctx):
    """Where FastMerging's scans over large core sets dominate the merge (a
    2M-point 3-D seed-spreader set at eps 2000: 619 core grids of about 3000
    core points, below the size that is merged by whole workgroups), the
    trained proposal makes the merge phase faster, at identical labels."""
    import paper_2210_07580_amd as G
    from paper_2210_07580_amd import proposal as P
    if not os.path.exists(P.BLOB_PATH):
        pytest.skip("no trained proposal committed")
    w = W.sweep_workload("simden", 3, eps=2000)
    t = torch.from_numpy(W.make_points(w).astype(np.float32)).cuda()
    merge, labels = {}, {}
    for name, blob in (("plain", None), ("learned", P.load_blob())):
        ctx.set_proposal(blob)
        try:
            labels[name] = ctx.dbscan(t, w.eps, w.minpts)
            ctx.set_option(G.GD_OPT_TIMING, 1)
            ms = []
            for _ in range(9):
                ctx.dbscan(t, w.eps, w.minpts)
                ms.append(ctx.phase_times()["merge"])
            merge[name] = float(np.median(ms))
        finally:
            ctx.set_option(G.GD_OPT_TIMING, 0)
            ctx.set_proposal(None)
    print(f"merge phase: plain {merge['plain']:.3f} ms, learned {merge['learned']:.3f} ms", flush=True)
    assert torch.equal(labels["plain"][0], labels["learned"][0])
    assert torch.equal(labels["plain"][1], labels["learned"][1])
    assert merge["learned"] < merge["plain"]
