"""400 million points in one call: every per-point array then passes 2^32
bytes (the input alone is 4.8 GB, the sorted rows 6.4 GB), so any 32-bit
offset or index product in the path would show, and its 84M grids take
kernels of one wave per grid past the 2^32 work-items a one-dimensional
launch can count.  The data are 20000 copies
of one 20000-point block (blobs plus noise, 1000 units wide) placed on a
lattice of pitch 1100, so that points of different copies are more than eps
apart.  DBSCAN (Definitions 1-5) then clusters each copy on its own, and
with canonical labels (smallest core index of a cluster) copy k's labels
are the block's plus k * 20000: the oracle clusters the block once and the
whole result is checked element by element against that."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS, MINPTS, PITCH, COPIES = 60, 12, 1100, 20000


@pytest.fixture(scope="module")
def G():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G


def block(seed=11, m=20000, extent=1000):
    rng = np.random.default_rng(seed)
    centres = rng.integers(100, extent - 100, size=(8, 3))
    x = centres[rng.integers(0, 8, size=m)] + rng.normal(0, 45, size=(m, 3))
    noise = rng.random(m) < 0.12
    x[noise] = rng.integers(0, extent, size=(noise.sum(), 3))
    return np.clip(np.rint(x), 0, extent).astype(np.int32)


def lattice(k, pitch):
    side = int(np.ceil(k ** (1 / 3)))
    i = np.arange(k)
    return np.stack([i % side, (i // side) % side, i // (side * side)], 1).astype(np.int32) * pitch


def test_four_hundred_million_points(G):
    b = block()
    m = len(b)
    n = COPIES * m
    free, _ = torch.cuda.mem_get_info()
    if free < 200 * 2**30:
        pytest.skip(f"needs about 200 GiB of free device memory, {free / 2**30:.0f} GiB free")
    want_l, want_c = oracle.dbscan(b, EPS, MINPTS)
    assert (want_l == -1).any() and ((want_l >= 0) & (want_c == 0)).any()
    off = torch.from_numpy(lattice(COPIES, PITCH)).cuda()
    x = (torch.from_numpy(b).cuda()[None] + off[:, None, :]).reshape(n, 3).float()
    del off
    print(f"case n={n} d=3 eps={EPS} minpts={MINPTS}, {free / 2**30:.0f} GiB free", flush=True)
    ctx = G.Context(0)
    lab, core = ctx.dbscan(x, EPS, MINPTS)
    torch.cuda.synchronize()
    st = ctx.stats()
    print(f"grids {st['grids']} key_bits {st['key_bits']}", flush=True)
    # more than 2^26 grids: a launch of one wave per grid passes 2^32
    # work-items, which a one-dimensional grid cannot count
    assert st["grids"] > 2**26
    del x
    wl = torch.from_numpy(want_l).cuda()
    base = (torch.arange(COPIES, device="cuda", dtype=torch.int32) * m)[:, None]
    exp = torch.where(wl[None] >= 0, wl[None] + base, torch.full_like(wl[None], -1))
    bad = (lab.view(COPIES, m) != exp).nonzero()
    assert bad.shape[0] == 0, f"{bad.shape[0]} labels differ, first (copy, point) {bad[:3].tolist()}"
    del exp, bad
    wc = torch.from_numpy(want_c).cuda()
    assert torch.equal(core.view(COPIES, m), wc[None].expand(COPIES, m)), "core flags differ"
    ctx.close()
    del lab, core
    torch.cuda.empty_cache()
