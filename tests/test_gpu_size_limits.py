"""The point-count bounds of the C ABI: one call takes 0 <= n < 2^31 and a
batch at most 2^31 - 1 points in all (sorted indices and labels are 32-bit).
Calls beyond them return GD_EINVAL before any device work; the pointers
passed are small real device buffers that the checks never read."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G


def test_counts_beyond_the_bounds_are_refused(G):
    lib = G.load_library()
    ctx = G.Context(0)
    pts = torch.zeros((4, 2), dtype=torch.float32, device="cuda")
    lab = torch.empty(4, dtype=torch.int32, device="cuda")
    core = torch.empty(4, dtype=torch.uint8, device="cuda")
    p, l, c = pts.data_ptr(), lab.data_ptr(), core.data_ptr()
    for entry in (lib.dbscan, lib.dbscan_noalloc):
        for n in (1 << 31, -1):
            assert entry(ctx._h, p, n, 2, 5.0, 2, l, c, None) == G.GD_EINVAL
            assert b"out of range" in lib.gd_last_error(ctx._h)
    # two instances of 2^30 points: 2^31 in all
    arr = (G.Instance * 2)()
    for k in range(2):
        arr[k].points, arr[k].n, arr[k].d, arr[k].minpts = p, 1 << 30, 2, 2
        arr[k].eps, arr[k].labels, arr[k].core_flags = 5.0, l, c
    assert lib.dbscan_batched(ctx._h, arr, 2, None) == G.GD_EINVAL
    assert b"batch holds" in lib.gd_last_error(ctx._h)
    # the context stays usable
    lab2, core2 = ctx.dbscan(pts, 5, 2)
    assert bool((core2 == 1).all()) and bool((lab2 == 0).all())
    ctx.close()
