"""Sorted coordinate rows rebuilt from bits carried through the sort
(GD_OPT_PACKED_ROWS).  With identifiers of 33-64 bits, or of up to 32 bits
whose grids are too wide for the 32-bit packed value, the low coordinate
bits ride in a 64-bit sort word below the identifier; the result must be the
oracle's and the same as with the rows gathered from the input, in single
calls, batches and graph replays, including a replay whose larger eps no
longer fits the captured bit width (that call must run eagerly instead)."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G


def clumps(seed, n, d, eps, half):
    """Clumps about an eps wide over [-half, half]^d, plus scattered points."""
    rng = np.random.default_rng(seed)
    centres = rng.integers(-half, half + 1, size=(max(1, n // 40), d))
    x = centres[rng.integers(0, len(centres), size=n)] + rng.integers(-eps, eps + 1, size=(n, d))
    x[: n // 8] = rng.integers(-half, half + 1, size=(n // 8, d))
    return np.clip(x, -half, half).astype(np.int32)


def run(ctx, x, eps, minpts):
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    lab, core = ctx.dbscan(t, eps, minpts)
    return lab.cpu().numpy(), core.cpu().numpy()


def same(got, want, what):
    assert np.array_equal(got[1], want[1]), f"{what}: core flags differ"
    bad = np.nonzero(got[0] != want[0])[0]
    assert bad.size == 0, f"{what}: {bad.size} labels differ, first at {bad[:5]}"


# (d, eps, half-extent): identifiers of 33-64 bits whose grids fit a few
# bits per coordinate beside them
CASES = [(3, 150, 50_000), (3, 40, 100_000), (2, 100, 1 << 23), (5, 20, 500), (3, 150, 200_000)]


@pytest.mark.parametrize("d,eps,half", CASES)
def test_two_word_identifiers_with_packed_rows(G, d, eps, half):
    x = clumps(700 + d + eps, 4000, d, eps, half)
    want = oracle.dbscan(x, eps, 5)
    for packed in (1, 0):
        ctx = G.Context(0)
        ctx.set_option(G.GD_OPT_PACKED_ROWS, packed)
        print(f"case d={d} eps={eps} half={half} packed={packed}", flush=True)
        same(run(ctx, x, eps, 5), want, f"packed={packed}")
        bits = ctx.stats()["key_bits"]
        assert 32 < bits <= 64, bits
        ctx.close()


# 32-bit identifiers whose grids are too wide for the 32-bit packed value:
# sorted as 64-bit words with the rows below them (the last also with eps
# above the 32-bit distance bound)
WIDE_CELLS = [(3, 2000, 50_000), (3, 5000, 200_000), (2, 100_000, 1 << 23)]


@pytest.mark.parametrize("d,eps,half", WIDE_CELLS)
def test_one_word_identifiers_of_wide_grids(G, d, eps, half):
    x = clumps(800 + d + eps, 4000, d, eps, half)
    want = oracle.dbscan(x, eps, 5)
    for packed in (1, 0):
        ctx = G.Context(0)
        ctx.set_option(G.GD_OPT_PACKED_ROWS, packed)
        print(f"case d={d} eps={eps} half={half} packed={packed}", flush=True)
        same(run(ctx, x, eps, 5), want, f"packed={packed}")
        assert ctx.stats()["key_bits"] <= 32
        ctx.close()


def test_bad_option_value(G):
    ctx = G.Context(0)
    with pytest.raises(G.GDError):
        ctx.set_option(G.GD_OPT_PACKED_ROWS, 3)
    ctx.close()


def test_batch_with_packed_rows_and_graph_replay(G):
    rng = np.random.default_rng(29)
    problems = []
    for k in range(10):
        d = int(rng.integers(2, 4))
        eps = int(rng.choice([60, 150, 300]))
        x = clumps(900 + k, int(rng.integers(0, 2500)), d, eps, 60_000)
        problems.append((x, eps, int(rng.integers(2, 9))))
    want = [oracle.dbscan(x, e, m) for x, e, m in problems]
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_GRAPH, 2)
    tens = [(torch.from_numpy(x.astype(np.float32)).cuda(), e, m) for x, e, m in problems]
    for rep in range(3):
        print(f"case batch call {rep}", flush=True)
        outs = ctx.dbscan_batched(tens)
        assert ctx.stats()["graph_replays"] == (1 if rep else 0)
        for k, ((lab, core), w) in enumerate(zip(outs, want)):
            same((lab.cpu().numpy(), core.cpu().numpy()), w, f"call {rep} instance {k}")
    ctx.close()


def test_replay_with_an_eps_beyond_the_captured_width(G):
    # eps 150 packs 7 bits per coordinate; eps 300 needs 8, so the replay of
    # the graph captured at 150 must be refused on the device and the call
    # run eagerly
    x = clumps(31, 5000, 3, 150, 200_000)
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_GRAPH, 2)
    for rep, eps in enumerate((150, 150, 300, 150)):
        print(f"case replay call {rep} eps {eps}", flush=True)
        lab, core = ctx.dbscan(t, eps, 4)
        same((lab.cpu().numpy(), core.cpu().numpy()), oracle.dbscan(x, eps, 4), f"call {rep} eps {eps}")
        assert 32 < ctx.stats()["key_bits"] <= 64
        if rep == 1:
            assert ctx.stats()["graph_replays"] == 1
    ctx.close()


# 32-bit identifiers with packed values: one instance rebuilds its rows in
# the sort's last pass (1), or in a pass of its own (2); batches always in a
# pass of their own
ONE_WORD = [(3, 200, 50_000), (2, 700, 1 << 20), (1, 50, 1 << 22), (4, 300, 5_000)]


@pytest.mark.parametrize("d,eps,half", ONE_WORD)
def test_rows_rebuilt_by_the_last_sort_pass(G, d, eps, half):
    x = clumps(600 + d + eps, 5000, d, eps, half)
    want = oracle.dbscan(x, eps, 5)
    for packed in (1, 2, 0):
        ctx = G.Context(0)
        ctx.set_option(G.GD_OPT_PACKED_ROWS, packed)
        print(f"case d={d} eps={eps} half={half} packed={packed}", flush=True)
        for rep in range(2):
            same(run(ctx, x, eps, 5), want, f"packed={packed} call {rep}")
        assert ctx.stats()["key_bits"] <= 32
        ctx.close()
