"""Contexts are independent: two host threads, each with its own context and
its own stream (one of them capturing and replaying graphs), cluster
different inputs at the same time, and every result must be the oracle's.
The library's only shared state, the allocation-free entry point's array
address, is looked up under a lock."""
import threading

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


def test_two_threads_with_their_own_contexts_and_streams(G):
    jobs = [
        [(W.WORKLOADS["cfg1"].with_n(100_000), None), (W.sweep_workload("varden", 5, n=40_000), 2000),
         (W.WORKLOADS["cfg0"], None)],
        [(W.WORKLOADS["H"].with_n(100_000), None), (W.sweep_workload("simden", 2, n=60_000), 3000),
         (W.WORKLOADS["cfg4"].with_n(80_000), None)],
    ]
    data = []
    for lane in jobs:
        items = []
        for w, eps in lane:
            x = W.make_points(w)
            e = eps or w.eps
            items.append((x, e, w.minpts, oracle.dbscan(x, e, w.minpts)))
        data.append(items)
    errors, results = [], [[None] * 3 for _ in range(2)]

    def work(t):
        try:
            ctx = G.Context(0)
            if t == 1:
                ctx.set_option(G.GD_OPT_GRAPH, 2)
            stream = torch.cuda.Stream()
            with torch.cuda.stream(stream):
                pts = [torch.from_numpy(x.astype(np.float32)).cuda() for x, _, _, _ in data[t]]
            stream.synchronize()
            # each input four times in a row: thread 1 captures on the first
            # call and replays the graph on the next three
            for i, (x, e, mp, _) in enumerate(data[t]):
                for rep in range(4):
                    lab, core = ctx.dbscan(pts[i], e, mp, stream=stream)
                    stream.synchronize()
                    if t == 1 and ctx.stats()["graph_replays"] != (1 if rep else 0):
                        errors.append(f"thread 1 input {i}: call {rep} did not {'replay' if rep else 'capture'}")
                    got = (lab.cpu().numpy(), core.cpu().numpy())
                    if results[t][i] is None:
                        results[t][i] = got
                    elif not (np.array_equal(got[0], results[t][i][0]) and np.array_equal(got[1], results[t][i][1])):
                        errors.append(f"thread {t} input {i}: call {rep} differs from call 0")
            ctx.close()
        except Exception as exc:  # reported by the main thread
            errors.append(f"thread {t}: {exc!r}")

    threads = [threading.Thread(target=work, args=(t,)) for t in range(2)]
    for th in threads:
        th.start()
    for th in threads:
        th.join(timeout=240)
    assert not any(th.is_alive() for th in threads), "a thread did not finish"
    assert not errors, errors
    for t in range(2):
        for i, (_, e, mp, (wl, wc)) in enumerate(data[t]):
            print(f"case thread {t} input {i} eps {e} minpts {mp}", flush=True)
            assert np.array_equal(results[t][i][1], wc), f"thread {t} input {i}: core flags"
            assert np.array_equal(results[t][i][0], wl), f"thread {t} input {i}: labels"
