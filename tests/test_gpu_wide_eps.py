"""eps above the 32-bit distance bound (GD_EPS_MAX = 21845): squared
distances are taken in 64 bits in every consumer.  Results must be the
oracle's on every dimension, in every merge order and neighbour mode, in
batches that mix both widths, across graph replays, with approximate
merging, and for the FastMerging test entry."""
import numpy as np
import pytest

import oracle
from oracle import steps

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LIM = 1 << 24


@pytest.fixture(scope="module")
def G():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G


def clustered(seed, n, d, eps):
    """Clumps a few eps wide, spread over a domain of about 40 eps (clipped
    to the valid coordinate range), plus scattered points."""
    rng = np.random.default_rng(seed)
    half = min(LIM, 20 * eps)
    centres = rng.integers(-half, half + 1, size=(max(1, n // 60), d))
    x = centres[rng.integers(0, len(centres), size=n)] + rng.integers(-eps, eps + 1, size=(n, d))
    x[: n // 10] = rng.integers(-half, half + 1, size=(n // 10, d))
    return np.clip(x, -LIM, LIM).astype(np.int32)


def run(ctx, x, eps, minpts):
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    lab, core = ctx.dbscan(t, eps, minpts)
    return lab.cpu().numpy(), core.cpu().numpy()


def same(got, want, what):
    assert np.array_equal(got[1], want[1]), f"{what}: core flags differ"
    bad = np.nonzero(got[0] != want[0])[0]
    assert bad.size == 0, f"{what}: {bad.size} labels differ, first at {bad[:5]}"


@pytest.mark.parametrize("seed", range(16))
def test_random_vs_brute(G, seed):
    rng = np.random.default_rng(600 + seed)
    d = 1 + seed % 8
    eps = int(rng.choice([21846, 30000, 65535, 65536, 250_000, 3_000_000]))
    n = int(rng.integers(1, 900))
    x = clustered(seed, n, d, eps)
    if n > 6:
        x[: n // 6] = x[n // 6: 2 * (n // 6)]  # duplicates
    minpts = int(rng.choice([1, 2, 3, 5, 9, 17, n + 1]))
    ctx = G.Context(0)
    print(f"case seed={seed} n={n} d={d} eps={eps} minpts={minpts}", flush=True)
    same(run(ctx, x, eps, minpts), oracle.dbscan_brute(x, eps, minpts), f"seed {seed}")
    ctx.close()


@pytest.mark.parametrize("eps", [2 ** 27, 2 ** 31, 10 ** 15])
def test_eps_beyond_every_distance(G, eps):
    # every pair of valid points is within 2^27: one cluster of core points
    # (MinPts <= n), whatever larger eps is asked for
    rng = np.random.default_rng(eps % 1000)
    x = rng.integers(-LIM, LIM + 1, size=(500, 8)).astype(np.int32)
    ctx = G.Context(0)
    lab, core = run(ctx, x, eps, 500)
    assert core.all() and (lab == 0).all()
    lab, core = run(ctx, x, eps, 501)
    assert (~core.astype(bool)).all() and (lab == -1).all()
    ctx.close()


@pytest.mark.parametrize("mode", ["ldf", "grid_order", "bfs", "walk", "lists_hash"])
@pytest.mark.parametrize("d", [2, 3, 5, 7])
def test_modes_vs_oracle(G, mode, d):
    eps = 40_000
    x = clustered(90 + d, 20_000, d, eps)
    want = oracle.dbscan(x, eps, 8)
    ctx = G.Context(0)
    if mode == "grid_order":
        ctx.set_option(G.GD_OPT_LDF_ORDER, 0)
    elif mode == "bfs":
        ctx.set_option(G.GD_OPT_MERGE_ORDER, 2)
    elif mode == "walk":
        ctx.set_option(G.GD_OPT_NEIGHBOR_MODE, 2)
    elif mode == "lists_hash":
        ctx.set_option(G.GD_OPT_NEIGHBOR_MODE, 1)
        ctx.set_option(G.GD_OPT_NEIGHBOR_QUERY, 2)
    ctx.set_option(G.GD_OPT_STATS, 1)
    print(f"case mode={mode} d={d}", flush=True)
    same(run(ctx, x, eps, 8), want, f"{mode} d={d}")
    st = ctx.stats()
    assert st["merge_pairs"] == st["merge_tests"] + st["merge_skipped"]
    ctx.close()


def test_batch_mixing_widths_and_graph_replay(G):
    rng = np.random.default_rng(17)
    problems = []
    for k in range(12):
        d = int(rng.integers(1, 6))
        eps = int(rng.choice([500, 9000, 21845, 21846, 60000]))
        x = clustered(200 + k, int(rng.integers(0, 1500)), d, eps)
        problems.append((x, eps, int(rng.integers(1, 10))))
    want = [oracle.dbscan(x, e, m) for x, e, m in problems]
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_GRAPH, 2)
    tens = [(torch.from_numpy(x.astype(np.float32)).cuda(), e, m) for x, e, m in problems]
    for rep in range(3):
        outs = ctx.dbscan_batched(tens)
        assert ctx.stats()["graph_replays"] == (1 if rep else 0)
        for k, ((lab, core), w) in enumerate(zip(outs, want)):
            same((lab.cpu().numpy(), core.cpu().numpy()), w, f"call {rep} instance {k}")
    ctx.close()


def test_replay_across_the_distance_bound(G):
    # captured with every eps on the 32-bit path; the same shape with an eps
    # above the bound must not replay the 32-bit kernels
    rng = np.random.default_rng(3)
    x = clustered(5, 3000, 2, 21000)
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_GRAPH, 2)
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    for rep, eps in enumerate((21000, 21000, 40000, 40000, 21000)):
        lab, core = ctx.dbscan(t, eps, 4)
        replayed = ctx.stats()["graph_replays"]
        assert replayed == (1 if rep in (1, 3) else 0), (rep, eps, replayed)
        same((lab.cpu().numpy(), core.cpu().numpy()), oracle.dbscan(x, eps, 4), f"call {rep} eps {eps}")
    del rng
    ctx.close()


def test_approximate_merge_with_wide_distances(G):
    eps, delta = 30_000, 3_000
    x = clustered(8, 4000, 3, eps)
    want_l, want_c = oracle.dbscan(x, eps, 6)
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_APPROX_DELTA, 0)
    same(run(ctx, x, eps, 6), (want_l, want_c), "delta 0")
    ctx.set_option(G.GD_OPT_APPROX_DELTA, delta)
    lab, core = run(ctx, x, eps, 6)
    assert np.array_equal(core, want_c)
    cm = want_c == 1
    relaxed = oracle.core_components(x, want_c, eps + delta)
    # exact clusters stay whole; joined clusters are within eps + delta
    for v in np.unique(want_l[cm]):
        assert np.unique(lab[cm & (want_l == v)]).size == 1
    for v in np.unique(lab[cm]):
        assert np.unique(relaxed[cm & (lab == v)]).size == 1
    ctx.close()


def test_merge_test_entry_with_wide_eps(G):
    rng = np.random.default_rng(12)
    d, eps = 3, 50_000
    m = 3000
    pts = rng.integers(-400_000, 400_000, size=(m, d)).astype(np.int32)
    pairs, want = [], []
    for _ in range(200):
        a0, b0 = (int(v) for v in rng.integers(0, m - 40, size=2))
        ac, bc = (int(v) for v in rng.integers(1, 40, size=2))
        pairs.append((a0, ac, b0, bc))
        want.append(steps.min_dist2(pts[a0:a0 + ac], pts[b0:b0 + bc]) <= eps * eps)
    ctx = G.Context(0)
    ans = ctx.merge_test(torch.from_numpy(np.ascontiguousarray(pts.T)).cuda(),
                         torch.tensor(pairs, dtype=torch.int32).cuda(), eps)
    got = ans.cpu().numpy()
    assert (got <= 1).all()
    assert got.astype(bool).tolist() == want
    assert 20 < sum(want) < len(want) - 20
    ctx.close()
