"""Core marking and the border search skip a neighbour grid whose cell lies
farther than eps from every query still open in the wave (d <= 4; core
marking does so in a kernel variant chosen when grids hold 1024 points or
more on average).  Cells of very uneven density side by side, with MinPts
near the 30th percentile of the neighbour counts, so that many queries stay
open across whole neighbourhoods: the result must be the oracle's."""
import math

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


def uneven_cells(seed, d, eps, shape, mean):
    """A block of `shape` cells of side eps / sqrt(d) (Eq. (1)), aligned to
    the grid by a point at the origin, each filled uniformly with a
    log-uniform share of points (the densest about 1000 times the sparsest),
    `mean` per cell on average."""
    rng = np.random.default_rng(seed)
    s = eps / math.sqrt(d)
    cells = np.stack(np.meshgrid(*[np.arange(m) for m in shape], indexing="ij"), -1).reshape(-1, d)
    w = np.exp(rng.uniform(np.log(2), np.log(2000), size=len(cells)))
    cnt = np.maximum(1, np.rint(w * mean / w.mean())).astype(int)
    c = np.repeat(cells, cnt, axis=0)
    lo = np.ceil(c * s)
    hi = np.ceil((c + 1) * s) - 1
    x = np.floor(lo + rng.random(lo.shape) * (hi - lo + 1)).astype(np.int32)
    x = x[rng.permutation(len(x))]
    x[0] = 0
    return x


def run(ctx, x, eps, minpts):
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
    lab, core = ctx.dbscan(t, eps, minpts)
    return lab.cpu().numpy(), core.cpu().numpy()


# (d, eps, cells per dimension, MinPts at about the 30th percentile of the
# neighbour counts, a low MinPts)
CASES = [(1, 1000, (40,), 4325, 300), (2, 2000, (8, 5), 5544, 500),
         (3, 3000, (4, 3, 2), 11482, 1000), (4, 3000, (3, 3, 2, 2), 20585, 2000)]


@pytest.mark.parametrize("d,eps,shape,minpts,low", CASES)
def test_pruned_neighbourhoods_match_the_oracle(G, d, eps, shape, minpts, low):
    x = uneven_cells(300 + d, d, eps, shape, 1150)
    ctx = G.Context(0)
    for mp in (minpts, low):
        want = oracle.dbscan(x, eps, mp)
        print(f"case d={d} eps={eps} n={len(x)} minpts={mp}", flush=True)
        for rep in range(2):
            lab, core = run(ctx, x, eps, mp)
            assert np.array_equal(core, want[1]), f"minpts {mp} call {rep}: core flags differ"
            bad = np.nonzero(lab != want[0])[0]
            assert bad.size == 0, f"minpts {mp} call {rep}: {bad.size} labels differ, first at {bad[:5]}"
        st = ctx.stats()
        # grids of 1024 points and more on average, as the data intend
        assert st["n"] >= 1024 * st["grids"], (st["n"], st["grids"])
        if mp == minpts:  # core and border points both
            assert 0 < want[1].sum() < len(x) and ((want[0] >= 0) & (want[1] == 0)).any()
    ctx.close()
