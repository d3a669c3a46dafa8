"""The sweep workloads (seed-spreader data in [0, 1e5]^d with similar or
variable density, d in {2, 3, 5, 7}; eps 500-5000, MinPts 10-100) at sizes
the oracle finishes quickly: bit-exact labels and core flags with both the
LDF order and the breadth-first searches of Algorithm 6.  At d = 7 and
eps = 500 the packed identifiers take two words."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctxs():
    import paper_2210_07580_amd as G
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    out = {}
    for order, v in (("ldf", 1), ("bfs", 2)):
        out[order] = G.Context(0)
        out[order].set_option(G.GD_OPT_MERGE_ORDER, v)
    yield out
    for c in out.values():
        c.close()


@pytest.mark.parametrize("kind", W.SWEEP_KINDS)
@pytest.mark.parametrize("d", W.SWEEP_DIMS)
def test_sweep_points_vs_oracle(ctxs, kind, d):
    w0 = W.sweep_workload(kind, d, n=30_000)
    x = W.make_points(w0)
    t = torch.from_numpy(x.astype(np.float32)).cuda()
    for eps, minpts in ((500, 100), (500, 10), (2000, 100), (5000, 100)):
        want_l, want_c = oracle.dbscan(x, eps, minpts)
        for order, ctx in ctxs.items():
            print(f"case {w0.name} eps={eps} minpts={minpts} order={order}", flush=True)
            lab, core = ctx.dbscan(t, eps, minpts)
            lab, core = lab.cpu().numpy(), core.cpu().numpy()
            assert np.array_equal(core, want_c), f"eps {eps} minpts {minpts} {order}: core flags"
            bad = np.nonzero(lab != want_l)[0]
            assert bad.size == 0, f"eps {eps} minpts {minpts} {order}: {bad.size} labels differ"
