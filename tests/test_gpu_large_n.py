"""400 million points in one call: every per-point array then passes 2^32
bytes (the input alone is 4.8 GB, the sorted rows 6.4 GB), so any 32-bit
offset or index product in the path would show, and the grids (84M of them
in blobs, 284M when sparse) take kernels of several lanes per grid past the
2^32 work-items a one-dimensional launch can count.  The data are 20000
copies of one 20000-point block placed on a lattice whose pitch exceeds the
block's width by more than eps, so that points of different copies are more
than eps apart.  DBSCAN (Definitions 1-5) then clusters each copy on its
own, and with canonical labels (smallest core index of a cluster) copy k's
labels are the block's plus k * 20000: the oracle clusters the block once
and the whole result is checked element by element against that."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

COPIES = 20000


@pytest.fixture(scope="module")
def G():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G


def block(seed=11, m=20000, extent=1000):
    """Eight blobs and 12% noise, 1000 units wide."""
    rng = np.random.default_rng(seed)
    centres = rng.integers(100, extent - 100, size=(8, 3))
    x = centres[rng.integers(0, 8, size=m)] + rng.normal(0, 45, size=(m, 3))
    noise = rng.random(m) < 0.12
    x[noise] = rng.integers(0, extent, size=(noise.sum(), 3))
    return np.clip(np.rint(x), 0, extent).astype(np.int32)


def sparse_block(seed=21, m=20000, extent=1790):
    """Uniform points at about 1.4 per grid of eps = 100 (a tenth of them in
    a denser corner), nearly all core at MinPts 5: hundreds of millions of
    tiny core grids once copied."""
    rng = np.random.default_rng(seed)
    x = rng.integers(0, extent + 1, size=(m, 3))
    x[: m // 10] = rng.integers(0, extent + 1, size=(m // 10, 3)) // 3
    return x.astype(np.int32)


def lattice(k, pitch):
    side = int(np.ceil(k ** (1 / 3)))
    i = np.arange(k)
    return np.stack([i % side, (i // side) % side, i // (side * side)], 1).astype(np.int32) * pitch


# (block, eps, MinPts, lattice pitch)
CASES = {"blobs": (block, 60, 12, 1100), "sparse": (sparse_block, 100, 5, 1900)}


# the learned proposal changes only the order of the merge's tests (its
# per-grid summaries launch past 2^32 work-items here too)
@pytest.mark.parametrize("kind,proposal", [("blobs", False), ("sparse", False), ("blobs", True)])
def test_four_hundred_million_points(G, kind, proposal):
    make, eps, minpts, pitch = CASES[kind]
    b = make()
    m = len(b)
    n = COPIES * m
    free, _ = torch.cuda.mem_get_info()
    if free < 200 * 2**30:
        pytest.skip(f"needs about 200 GiB of free device memory, {free / 2**30:.0f} GiB free")
    want_l, want_c = oracle.dbscan(b, eps, minpts)
    assert want_c.any() and ((want_l >= 0) & (want_c == 0)).any()
    off = torch.from_numpy(lattice(COPIES, pitch)).cuda()
    x = (torch.from_numpy(b).cuda()[None] + off[:, None, :]).reshape(n, 3).float()
    del off
    print(f"case {kind} n={n} d=3 eps={eps} minpts={minpts}, {free / 2**30:.0f} GiB free", flush=True)
    ctx = G.Context(0)
    if proposal:
        from paper_2210_07580_amd import proposal as P
        ctx.set_proposal(P.load_blob())
    lab, core = ctx.dbscan(x, eps, minpts)
    torch.cuda.synchronize()
    st = ctx.stats()
    print(f"grids {st['grids']} core grids {st['core_grids']} entries {st['neighbor_entries']}", flush=True)
    # more than 2^26 grids: a launch of one wave per grid passes 2^32
    # work-items, which a one-dimensional grid cannot count
    assert st["grids"] > 2**26
    if kind == "sparse":  # the tiny-set merge too, and lists past 2^32 entries
        assert st["core_grids"] > 2**26 and st["neighbor_entries"] > 2**32
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


def test_batch_of_four_hundred_million_points(G):
    """Ten instances of 40M points each (2000 blob copies, each instance
    shifted) in one batched call, then again as a graph replay: every
    instance's labels are the block's shifted by the copy's first index
    within that instance."""
    free, _ = torch.cuda.mem_get_info()
    if free < 200 * 2**30:
        pytest.skip(f"needs about 200 GiB of free device memory, {free / 2**30:.0f} GiB free")
    make, eps, minpts, pitch = CASES["blobs"]
    b = make()
    m = len(b)
    want_l, want_c = oracle.dbscan(b, eps, minpts)
    inst, k = 10, 2000
    off = torch.from_numpy(lattice(k, pitch)).cuda()
    xs = [((torch.from_numpy(b).cuda()[None] + off[:, None, :]).reshape(k * m, 3) + 7 * i).float() for i in range(inst)]
    del off
    wl = torch.from_numpy(want_l).cuda()
    wc = torch.from_numpy(want_c).cuda()
    base = (torch.arange(k, device="cuda", dtype=torch.int32) * m)[:, None]
    exp = torch.where(wl[None] >= 0, wl[None] + base, torch.full_like(wl[None], -1))
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_GRAPH, 1)
    for rep in range(2):
        print(f"case batch of {inst} x {k * m} points, call {rep}", flush=True)
        outs = ctx.dbscan_batched([(x, eps, minpts) for x in xs])
        torch.cuda.synchronize()
        st = ctx.stats()
        assert st["graph_replays"] == rep and st["grids"] > 2**26
        for i, (lab, core) in enumerate(outs):
            assert torch.equal(lab.view(k, m), exp), f"call {rep} instance {i}: labels differ"
            assert torch.equal(core.view(k, m), wc[None].expand(k, m)), f"call {rep} instance {i}: core flags differ"
        del outs
    ctx.close()
    del xs
    torch.cuda.empty_cache()


def blobs_d(seed, m, d, extent, sigma, k=12, noise=0.1):
    """k Gaussian blobs plus uniform noise in [0, extent]^d."""
    rng = np.random.default_rng(seed)
    centres = rng.integers(int(3 * sigma), extent - int(3 * sigma), size=(k, d))
    x = centres[rng.integers(0, k, size=m)] + rng.normal(0, sigma, size=(m, d))
    nz = rng.random(m) < noise
    x[nz] = rng.integers(0, extent, size=(nz.sum(), d))
    return np.clip(np.rint(x), 0, extent).astype(np.int32)


def lattice_d(k, d, pitch):
    side = 1
    while side ** d < k:
        side += 1
    i = np.arange(k)
    return np.stack([(i // side ** j) % side for j in range(d)], 1).astype(np.int32) * pitch


# d = 8 with identifiers of 72 bits (two words; 100M grids, 1.9e10 neighbour
# entries) and d = 1 (copies along one axis up to 1.6e7, below 2^24)
OTHER = {"d8_two_words": (dict(seed=5, m=20000, d=8, extent=1000, sigma=12), 20, 5, 1100, 64),
         "d1": (dict(seed=6, m=20000, d=1, extent=2800, sigma=3, k=20, noise=0.3), 2, 20, 3000, 0)}


@pytest.mark.parametrize("kind", sorted(OTHER))
def test_hundred_million_points_at_d8_and_d1(G, kind):
    kw, eps, minpts, pitch, min_bits = OTHER[kind]
    copies = 5000
    free, _ = torch.cuda.mem_get_info()
    if free < 200 * 2**30:
        pytest.skip(f"needs about 200 GiB of free device memory, {free / 2**30:.0f} GiB free")
    b = blobs_d(**kw)
    m, d = b.shape
    want_l, want_c = oracle.dbscan(b, eps, minpts)
    assert want_c.any() and (want_l == -1).any() and ((want_l >= 0) & (want_c == 0)).any()
    off = torch.from_numpy(lattice_d(copies, d, pitch)).cuda()
    x = (torch.from_numpy(b).cuda()[None] + off[:, None, :]).reshape(copies * m, d).float()
    del off
    print(f"case {kind} n={copies * m} d={d} eps={eps} minpts={minpts}", flush=True)
    ctx = G.Context(0)
    lab, core = ctx.dbscan(x, eps, minpts)
    torch.cuda.synchronize()
    assert ctx.stats()["key_bits"] > min_bits
    del x
    wl = torch.from_numpy(want_l).cuda()
    base = (torch.arange(copies, device="cuda", dtype=torch.int32) * m)[:, None]
    exp = torch.where(wl[None] >= 0, wl[None] + base, torch.full_like(wl[None], -1))
    assert torch.equal(lab.view(copies, m), exp), "labels differ"
    wc = torch.from_numpy(want_c).cuda()
    assert torch.equal(core.view(copies, m), wc[None].expand(copies, m)), "core flags differ"
    ctx.close()
    del lab, core, exp
    torch.cuda.empty_cache()


def test_degenerate_inputs_at_scale(G):
    """Closed-form cases: 100M identical points (one grid); 100M points on
    two spots 1e6 apart; a chain of 2^24 points one unit apart in shuffled
    input order at eps 1, MinPts 3 (16.8M grids merged end to end: the two
    ends are border points, the rest core, one cluster named by the
    smallest input index of an interior point); 50M points over the whole
    accepted range [-2^24, 2^24]^2 at eps 2^28 (one grid, one cluster)."""
    ctx = G.Context(0)
    n = 100_000_000
    x = torch.zeros((n, 3), device="cuda")
    lab, core = ctx.dbscan(x, 5, 10)
    assert bool((core == 1).all()) and bool((lab == 0).all()) and ctx.stats()["grids"] == 1
    x[n // 2:, 0] = 1e6
    lab, core = ctx.dbscan(x, 5, 10)
    assert bool((core == 1).all()) and bool((lab[: n // 2] == 0).all()) and bool((lab[n // 2:] == n // 2).all())
    del x, lab, core
    m = 1 << 24
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    perm = torch.randperm(m, device="cuda", generator=g)
    x = perm.float().view(m, 1) - (1 << 23)
    lab, core = ctx.dbscan(x, 1, 3)
    interior = (perm != 0) & (perm != m - 1)
    assert torch.equal(core.bool(), interior)
    assert bool((lab == int(torch.nonzero(interior)[0])).all())
    assert ctx.stats()["grids"] == m
    del x, lab, core, perm, interior
    x = (torch.rand((50_000_000, 2), device="cuda", generator=g) * 2**25 - 2**24).round().clamp(-2**24, 2**24)
    lab, core = ctx.dbscan(x, 2**28, 7)
    assert bool((core == 1).all()) and bool((lab == 0).all())
    ctx.close()
    del x, lab, core
    torch.cuda.empty_cache()
