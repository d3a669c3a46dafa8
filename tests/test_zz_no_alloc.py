"""dbscan_noalloc: the entry point that takes every workspace buffer from
the library's fixed per-device scratch array.  Its output must equal
dbscan()'s bit for bit (and the oracle's), on consecutive calls whose inputs
shrink, and inputs beyond the array must be refused with a clear error."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def G():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return G


def _cases():
    # a larger call, then smaller ones: the scratch keeps the previous call's
    # contents, so whatever must start at zero has to be cleared by the call
    return [("cfg1", 300_000), ("H", 120_000), ("cfg0", 10_000), ("cfg0", 2_500)]


def test_noalloc_equals_dbscan_on_shrinking_calls(G):
    ctx = G.Context(0)
    ref = G.Context(0)
    for name, n in _cases():
        w = W.WORKLOADS[name]
        x = W.make_points(w, n=n)
        t = torch.from_numpy(x.astype(np.float32)).cuda()
        print(f"case: {name} n={n} d={w.d} eps={w.eps} minpts={w.minpts}", flush=True)
        lab = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        core = torch.full((n,), 9, dtype=torch.uint8, device="cuda")
        ctx.dbscan_noalloc(t, w.eps, w.minpts, lab, core)
        rl, rc = ref.dbscan(t, w.eps, w.minpts)
        assert torch.equal(core, rc), f"{name}@{n}: core flags differ from dbscan()"
        assert torch.equal(lab, rl), f"{name}@{n}: labels differ from dbscan()"
        if n <= 120_000:
            wl, wc = oracle.dbscan(x, w.eps, w.minpts)
            assert np.array_equal(core.cpu().numpy(), wc) and np.array_equal(lab.cpu().numpy(), wl)
    ctx.close()
    ref.close()


def test_noalloc_two_contexts_share_the_array_serially(G):
    # two contexts on one device use the same array; serial calls are fine
    a, b = G.Context(0), G.Context(0)
    w = W.WORKLOADS["cfg0"]
    x = W.make_points(w)
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    want_l, want_c = oracle.dbscan(x, w.eps, w.minpts)
    for c in (a, b, a):
        lab = torch.empty(len(x), dtype=torch.int32, device="cuda")
        core = torch.empty(len(x), dtype=torch.uint8, device="cuda")
        c.dbscan_noalloc(t, w.eps, w.minpts, lab, core)
        assert np.array_equal(core.cpu().numpy(), want_c) and np.array_equal(lab.cpu().numpy(), want_l)
    a.close()
    b.close()


def test_noalloc_refuses_inputs_beyond_the_array(G):
    ctx = G.Context(0)
    n = 3_000_000  # at d = 8 the workspace alone is far above 256 MiB
    x = torch.zeros((n, 8), dtype=torch.float32, device="cuda")
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    core = torch.empty(n, dtype=torch.uint8, device="cuda")
    print("case: n=3M d=8 (over the scratch size)", flush=True)
    with pytest.raises(G.GDError) as e:
        ctx.dbscan_noalloc(x, 10, 5, lab, core)
    assert e.value.status == G.GD_ENOMEM and "scratch" in str(e.value)
    # the context still works afterwards, with and without the scratch
    w = W.WORKLOADS["cfg0"]
    y = torch.from_numpy(W.make_points(w).astype(np.float32)).cuda()
    l2 = torch.empty(len(y), dtype=torch.int32, device="cuda")
    c2 = torch.empty(len(y), dtype=torch.uint8, device="cuda")
    ctx.dbscan_noalloc(y, w.eps, w.minpts, l2, c2)
    rl, rc = ctx.dbscan(y, w.eps, w.minpts)
    assert torch.equal(l2, rl) and torch.equal(c2, rc)
    ctx.close()
