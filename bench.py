#!/usr/bin/env python
"""Throughput of exact grid DBSCAN on one MI355X.

One step = one dbscan() call over the whole workload (every phase of the
hot path: identifiers, radix sort, grids, grid tree, neighbour lists, core
marking, FastMerging + union-find, labels, border assignment, output), with
the points already resident in device memory.  Prints one JSON line.

The K timed steps run the plain call; per-phase durations (for the
rooflines) come from K more steps with HIP events around every phase.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload H]
    python bench.py --sweep FILE [--sweep-dims 2,3,5,7] [--sweep-kinds simden,varden]
                    [--sweep-axes eps,minpts,n]

--sweep runs the paper's parameter sweeps (running time against eps, MinPts
and n on seed-spreader data) instead, writes one JSON record per sweep point
to FILE and prints a one-line summary.
"""
import argparse
import json
import os
import math
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0

WORKLOAD_DESC = {
    "H": "seed-spreader n=10M d=3 eps=200 minpts=100 (100 pts/step, radius 100, step 50, restart 0.001, 0.01% noise)",
    "cfg1": "seed-spreader n=2M d=3 eps=200 minpts=100",
    "cfg2": "gaussian blobs n=10M d=5 eps=5000 minpts=20 (100 blobs, sigma 2000-20000, 1% noise)",
    "cfg4": "seed-spreader n=20M d=3 eps=150 minpts=50 (300 pts/step)",
    "cfg0": "gaussian blobs n=10k d=2 eps=100 minpts=10",
}


# The kernels each timed phase launches (a phase is the run of launches
# between two events; the kernel traces under profiles/ list them one by one).
PHASE_KERNELS = {
    "minmax": ["minmax_kernel", "minmax_finish_kernel", "layout_kernel (batches of several instances)"],
    "keys": ["keys_kernel"],
    "radix_sort": ["per pass: radix_hist_kernel", "scan_reduce_kernel", "scan_down_kernel", "radix_scatter_kernel "
                   "(one instance with packed values: the last pass also writes the sorted rows)"],
    "gather": ["unpack_kernel or unpack64_kernel (rows rebuilt in order; gather_kernel when the low bits do "
               "not fit)"],
    "core_mark": ["core_mark_kernel"],
    "merge": ["merge_small_kernel", "merge_big_kernel"],
    "output": ["hash_clear_kernel", "hash_build_kernel", "output_direct_kernel", "output_kernel"],
    "nei_fill": ["nei_fill_kernel"],
}


def packed_rows(d, eps, key_bits):
    """How the library rebuilds the sorted rows of one instance (its pack_fits
    and pack64_bits rules): "value" (32-bit identifiers, the low coordinate
    bits in the 64-bit sort value beside the index), "word" (the low bits
    below the identifier in a 64-bit sort word, the index as the value), or
    None (the rows gathered from the input)."""
    fits = lambda bits: eps / math.sqrt(d) + 4.0 < 2.0 ** bits
    if key_bits <= 32 and fits(32 // d):
        return "value"
    b = next((bits for bits in range(1, 32) if fits(bits)), 0)
    return "word" if b and key_bits + d * b <= 64 else None


def algorithmic_bytes(phase, n, d, st, key_bytes, passes, packed):
    """Bytes the phase must move at least (the method's own traffic), per
    call; key_bytes: the sort word (8 with packed == "word").  A single
    instance with packed values ("value") has its rows written by the sort's
    last pass (no row phase of its own)."""
    B = 4 * d  # coordinates per point
    V = 8 if packed == "value" else 4  # sort value: index, with the packed low bits
    if phase == "minmax":
        return n * B
    if phase == "keys":
        return n * (B + key_bytes + (8 if packed == "value" else 0))
    if phase == "radix_sort":
        # per pass: histogram read of the keys, then (key, value) read and
        # written; with "value" the last pass writes the row and the index
        # instead of the value
        fused = n * (B + 4 - V) if packed == "value" and passes > 0 else 0
        return passes * n * (key_bytes + 2 * (key_bytes + V)) + fused
    if phase == "gather":
        # "value": sorted keys and values in, index and rows out; "word": the
        # words in, rows and identifiers out; else the index, one row in and
        # one row out
        if packed == "value":
            return n * (key_bytes + 8 + 4 + B)
        if packed == "word":
            return n * (2 * key_bytes + B)
        return n * (4 + 2 * B)
    if phase == "core_mark":
        # flags, plus every neighbour point streamed for a sparse grid (8 B per neighbour grid opened)
        return n + st["core_candidates"] * B + 8 * st["core_neighbor_grids"]
    if phase == "merge":
        # each tested pair reads both core sets once (+ 16 B of grid metadata)
        return st["merge_set_points"] * B + 16 * st["merge_tests"]
    if phase == "output":
        return n * (4 + 4 + 1)
    if phase == "nei_fill":
        return st["neighbor_entries"] * 4 + st["grids"] * (8 + 4 * d)
    return None


def source_digest():
    """SHA-256 of the HIP sources: counter-based traffic figures are only
    reported for the kernels they were taken from."""
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2210_07580_amd", "csrc")
    for name in sorted(os.listdir(src)):
        if name.endswith((".hip", ".hpp")):
            h.update(name.encode())
            with open(os.path.join(src, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per call and phase from the committed hardware-counter
    summary of this workload, if it was taken from the current sources."""
    import glob
    import re
    for path in glob.glob(os.path.join(ROOT, "profiles", "pmc_traffic_*.md")):
        with open(path) as f:
            text = f.read()
        m = re.search(r"```json\n(.*?)\n```", text, re.S)
        if not m:
            continue
        rec = json.loads(m.group(1))
        if rec.get("workload") == workload and rec.get("source_sha256") == source_digest():
            return rec.get("phases", {})
    return {}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_cpu():
    """Model name and clock of the host cores (from /proc/cpuinfo)."""
    model, mhz = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and model is None:
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("cpu MHz") and mhz is None:
                    mhz = float(line.split(":", 1)[1])
    except OSError:
        pass
    return {"model": model, "mhz": mhz, "logical_cpus": os.cpu_count()}


def cpu_baseline(w, sample_n):
    import oracle
    x = W.make_points(w, n=sample_n)
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.dbscan(x, w.eps, w.minpts, nthreads=threads)
    dt = time.perf_counter() - t0
    # the small blob workload whole, on all threads and on one
    w0 = W.WORKLOADS["cfg0"]
    x0 = W.make_points(w0)
    single = {}
    for th in (threads, 1):
        t1 = time.perf_counter()
        oracle.dbscan(x0, w0.eps, w0.minpts, nthreads=th)
        single[th] = time.perf_counter() - t1
    return {
        "value": round(sample_n / dt, 1),
        "unit": "points/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"the same generator ({w.name}) at n={sample_n:,}: same density recipe, full oracle "
                   f"clustering (eps-side cells, pointwise range queries, union-find), {dt:.1f} s"),
        "host": host_cpu(),
        "cfg0_whole": {"n": int(x0.shape[0]), "seconds_all_threads": round(single[threads], 4),
                       "seconds_one_thread": round(single[1], 4),
                       "one_thread_points_per_s": round(x0.shape[0] / single[1], 1)},
    }


_POINTS = {}


def points(name):
    """Device tensor of a workload's points (generated once per run)."""
    import torch
    if name not in _POINTS:
        w = W.WORKLOADS[name]
        log(f"bench: generating {w.name} n={w.n:,} d={w.d}")
        _POINTS[name] = torch.from_numpy(W.make_points(w).astype(np.float32)).cuda()
    return _POINTS[name]


def oracle_digest(name):
    """Stored SHA-256 digests of the oracle's labels and core flags for a
    workload (tests/golden/oracle_digests.json), or None."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_digests.json")
    try:
        with open(path) as f:
            rec = json.load(f).get(name)
    except OSError:
        return None
    return rec if isinstance(rec, dict) else None


def matches_oracle(name, lab, core):
    import hashlib
    rec = oracle_digest(name)
    if rec is None:
        return None
    sl = hashlib.sha256(np.ascontiguousarray(lab.cpu().numpy().astype("<i4")).tobytes()).hexdigest()
    sc = hashlib.sha256(np.ascontiguousarray(core.cpu().numpy().astype(np.uint8)).tobytes()).hexdigest()
    return sl == rec["labels_sha256"] and sc == rec["core_sha256"]


def run_plain(G, name, steps, warmup, options=(), blob=None):
    """One workload with the plain call (the learned proposal set when a blob
    is given): wall time per call, phase times, work counters, and the labels."""
    import torch
    w = W.WORKLOADS[name]
    pts = points(name)
    n = int(pts.shape[0])
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    core = torch.empty(n, dtype=torch.uint8, device="cuda")
    ctx = G.Context(0)
    for opt, val in options:
        ctx.set_option(opt, val)
    if blob is not None:
        ctx.set_proposal(blob)
    ms = []
    for i in range(warmup + steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.dbscan(pts, w.eps, w.minpts, lab, core)
        if i >= warmup:
            ms.append(1e3 * (time.perf_counter() - t0))
    ctx.set_option(G.GD_OPT_TIMING, 1)
    ctx.dbscan(pts, w.eps, w.minpts, lab, core)
    phases = {k: round(v, 4) for k, v in ctx.phase_times().items() if v > 0}
    ctx.set_option(G.GD_OPT_TIMING, 0)
    ctx.set_option(G.GD_OPT_STATS, 1)
    ctx.dbscan(pts, w.eps, w.minpts, lab, core)
    st = ctx.stats()
    ctx.close()
    med = float(np.median(ms))
    return {"n": n, "d": w.d, "eps": w.eps, "minpts": w.minpts, "value": round(n / (med * 1e-3), 1),
            "ms_median": round(med, 3), "ms_min": round(min(ms), 3), "ms_max": round(max(ms), 3),
            "phases_ms": phases, "labels": (lab, core), "stats": st}


def bench_configs(G, steps, warmup):
    """Plain points/s of the listed configurations beside the headline."""
    out = {}
    for name in ("cfg0", "cfg1", "cfg2"):
        r = run_plain(G, name, steps, warmup)
        lab, core = r.pop("labels")
        st = r.pop("stats")
        r["workload"] = WORKLOAD_DESC[name]
        r["labels_equal_oracle_digest"] = matches_oracle(name, lab, core)
        r["work"] = {k: st[k] for k in ("grids", "neighbor_entries", "core_points", "core_grids", "merge_tests",
                                        "merge_distances", "core_distances", "neighbor_walk")}
        out[name] = r
        log(f"bench: {name} {r['ms_median']} ms ({r['value']:.3g} points/s)")
    return out


def bench_merge_orders(G, steps, warmup):
    """Merge-order ablation (grid order, LDF, the BFS searches of Algorithm 6,
    LDF with the learned proposal): work and merge time at identical labels."""
    import torch
    from paper_2210_07580_amd import proposal as P
    orders = {"grid": [(G.GD_OPT_MERGE_ORDER, 0)], "ldf": [(G.GD_OPT_MERGE_ORDER, 1)],
              "bfs": [(G.GD_OPT_MERGE_ORDER, 2)], "learned": [(G.GD_OPT_MERGE_ORDER, 1), ("proposal", 1)]}
    out = {}
    for name in ("cfg1", "H", "cfg4"):
        res, ref = {}, None
        for oname, opts in orders.items():
            plain = [o for o in opts if o[0] != "proposal"]
            blob = P.load_blob() if any(o[0] == "proposal" for o in opts) else None
            r = run_plain(G, name, steps, warmup, plain, blob)
            lab, core = r.pop("labels")
            st = r.pop("stats")
            if ref is None:
                ref = (lab.clone(), core.clone())
            elif not (torch.equal(ref[0], lab) and torch.equal(ref[1], core)):
                raise RuntimeError(f"merge order {oname} changed the labels on {name}")
            res[oname] = {"ms_median": r["ms_median"], "merge_ms": r["phases_ms"].get("merge", 0.0),
                          "ldf_order_ms": r["phases_ms"].get("ldf_order", 0.0),
                          **{k: st[k] for k in ("merge_pairs", "merge_skipped", "merge_tests", "merge_yes",
                                                "merge_iterations", "merge_distances")}}
            log(f"bench: merge order {oname} on {name}: {res[oname]}")
        out[name] = res
    return out


def bench_approx(G, steps, warmup):
    """Approximate FastMerging (a yes once a pair within eps + delta is met)
    against the exact merge: time, iterations and how the clusters differ."""
    import torch
    out = {}
    for name in ("H", "cfg4"):
        w = W.WORKLOADS[name]
        res, exact = {}, None
        for delta in (0, w.eps // 10, w.eps // 2):
            r = run_plain(G, name, steps, warmup, [(G.GD_OPT_APPROX_DELTA, delta)])
            lab, core = r.pop("labels")
            st = r.pop("stats")
            clusters = int(torch.unique(lab[lab >= 0]).numel())
            if exact is None:
                exact = lab.clone()
            res[f"delta_{delta}"] = {
                "ms_median": r["ms_median"], "merge_ms": r["phases_ms"].get("merge", 0.0),
                "merge_tests": st["merge_tests"], "merge_iterations": st["merge_iterations"],
                "merge_max_iterations": st["merge_max_iterations"], "merge_distances": st["merge_distances"],
                "clusters": clusters, "labels_equal_exact": bool(torch.equal(lab, exact))}
            log(f"bench: approximate merge on {name}, delta {delta}: {res[f'delta_{delta}']}")
        out[name] = res
    return out


def bench_neighbor_modes(G, steps, warmup):
    """Neighbour-query ablation at identical labels: lists written for every
    grid by the grid tree (offset order; walk order above 2^20 grids), the
    grid tree in walk order (no offset order for early exit), direct hashing
    of every candidate identifier, and the consumers walking the grid tree
    themselves (no lists).  Hashing is left out for the 5-D workload, where
    every grid probes 3902 candidate identifiers."""
    import torch
    variants = {"tree_lists": [(G.GD_OPT_NEIGHBOR_MODE, 1), (G.GD_OPT_NEIGHBOR_QUERY, 3)],
                "tree_lists_walk_order": [(G.GD_OPT_NEIGHBOR_MODE, 1), (G.GD_OPT_NEIGHBOR_QUERY, 1)],
                "hash_lists": [(G.GD_OPT_NEIGHBOR_MODE, 1), (G.GD_OPT_NEIGHBOR_QUERY, 2)],
                "tree_walks_in_consumers": [(G.GD_OPT_NEIGHBOR_MODE, 2)]}
    out = {}
    for name in ("H", "cfg1", "cfg2"):
        res, ref = {}, None
        for vname, opts in variants.items():
            if name == "cfg2" and vname == "hash_lists":
                continue
            r = run_plain(G, name, steps, warmup, opts)
            lab, core = r.pop("labels")
            st = r.pop("stats")
            if ref is None:
                ref = (lab.clone(), core.clone())
            elif not (torch.equal(ref[0], lab) and torch.equal(ref[1], core)):
                raise RuntimeError(f"neighbour query {vname} changed the labels on {name}")
            ph = r["phases_ms"]
            res[vname] = {"ms_median": r["ms_median"], "nei_count_ms": ph.get("nei_count", 0.0),
                          "nei_fill_ms": ph.get("nei_fill", 0.0), "core_mark_ms": ph.get("core_mark", 0.0),
                          "merge_ms": ph.get("merge", 0.0), "output_ms": ph.get("output", 0.0),
                          "neighbor_entries": st["neighbor_entries"], "core_neighbor_grids": st["core_neighbor_grids"],
                          "core_candidates": st["core_candidates"]}
            log(f"bench: neighbour query {vname} on {name}: {r['ms_median']} ms")
        out[name] = res
    return out


def time_calls(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def bench_batched(G, steps, warmup, max_instances):
    """The 256-instance workload: one dbscan_batched() call versus one
    dbscan() call per instance, same GPU, identical results."""
    import torch
    ws = W.batch_workloads()[:max_instances]
    log(f"bench: generating {len(ws)} batch instances")
    probs = []
    for w in ws:
        x = W.make_points(w)
        probs.append((torch.from_numpy(x.astype(np.float32)).cuda(), w.eps, w.minpts))
    total = sum(int(p[0].shape[0]) for p in probs)
    ctx = G.Context(0)
    tuned, trials = ctx.autotune(probs)
    log(f"bench: autotuned {tuned}")
    outs = ctx.dbscan_batched(probs)
    for (t, e, m), (lab, core) in zip(probs[:8], outs[:8]):
        l1, c1 = ctx.dbscan(t, e, m)
        if not (torch.equal(l1, lab) and torch.equal(c1, core)):
            raise RuntimeError("batched and single-instance results differ")
    t_batch = time_calls(lambda: ctx.dbscan_batched(probs, outs=outs), steps, warmup)
    replayed = ctx.stats()["graph_replays"] == 1
    log(f"bench: batched {1e3 * t_batch:.2f} ms (graph replay: {replayed})")
    ctx.set_option(G.GD_OPT_GRAPH, 0)
    t_batch_eager = time_calls(lambda: ctx.dbscan_batched(probs, outs=outs), steps, warmup)
    log(f"bench: batched without graph {1e3 * t_batch_eager:.2f} ms")
    ctx.set_option(G.GD_OPT_TIMING, 1)
    ctx.dbscan_batched(probs, outs=outs)
    batch_phases = {k: round(v, 4) for k, v in ctx.phase_times().items()}
    ctx.set_option(G.GD_OPT_TIMING, 0)
    ctx.set_option(G.GD_OPT_STATS, 1)
    ctx.dbscan_batched(probs, outs=outs)
    bst = ctx.stats()
    ctx.set_option(G.GD_OPT_STATS, 0)

    def each():
        for (t, e, m), (lab, core) in zip(probs, outs):
            ctx.dbscan(t, e, m, lab, core)
    t_each = time_calls(each, max(1, steps // 2), 1)
    log(f"bench: one call per instance {1e3 * t_each:.2f} ms")
    ctx.close()
    return {
        "workload": f"{len(ws)} instances: n log-uniform [1e3,1e6], d in {{2,3}}, gaussian blobs + 10% noise, "
                    "eps in [50,300], minpts in [5,50]",
        "instances": len(ws), "points": total,
        "value": round(total / t_batch, 1), "ms_per_batch": round(1e3 * t_batch, 3),
        "plain_value": round(total / t_each, 1), "plain_ms_per_batch": round(1e3 * t_each, 3),
        "speedup_vs_plain": round(t_each / t_batch, 3), "unit": "points/s",
        "autotuned": tuned,
        "autotune_trials_ms": {f"tile{r['tile_points']}_waves{r['merge_waves']}_lanes{r['grid_lanes']}":
                               round(r["ms"], 3) for r in trials},
        "autotune_spread": round(max(r["ms"] for r in trials) / min(r["ms"] for r in trials), 3) if trials else None,
        "graph_replay": replayed, "no_graph_value": round(total / t_batch_eager, 1),
        "no_graph_ms_per_batch": round(1e3 * t_batch_eager, 3), "phases_ms": batch_phases,
        "work": {k: bst[k] for k in ("grids", "neighbor_entries", "core_points", "core_grids", "merge_tests",
                                     "merge_distances", "core_distances", "key_bits")},
    }


def learned_pair(G, pts, eps, minpts, steps, warmup):
    """Plain merge versus the trained proposal on one point set: call time,
    merge-phase time and merge work, at identical labels."""
    import torch
    from paper_2210_07580_amd import proposal as P
    n = int(pts.shape[0])
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    core = torch.empty(n, dtype=torch.uint8, device="cuda")
    ctx = G.Context(0)
    res = {}
    ref = None
    for name, blob in (("plain", None), ("learned", P.load_blob())):
        ctx.set_proposal(blob)
        t = time_calls(lambda: ctx.dbscan(pts, eps, minpts, lab, core), steps, warmup)
        # the merge phase alone, from calls with phase events
        ctx.set_option(G.GD_OPT_TIMING, 1)
        merge_ms = []
        for _ in range(steps):
            ctx.dbscan(pts, eps, minpts, lab, core)
            merge_ms.append(ctx.phase_times()["merge"])
        ctx.set_option(G.GD_OPT_TIMING, 0)
        ctx.set_option(G.GD_OPT_STATS, 1)
        ctx.dbscan(pts, eps, minpts, lab, core)
        st = ctx.stats()
        ctx.set_option(G.GD_OPT_STATS, 0)
        out = (lab.clone(), core.clone())
        if ref is None:
            ref = out
        elif not (torch.equal(ref[0], out[0]) and torch.equal(ref[1], out[1])):
            raise RuntimeError("learned proposal changed the labels")
        res[name] = {"value": round(n / t, 1), "ms_per_step": round(1e3 * t, 3),
                     "merge_ms": round(float(np.median(merge_ms)), 4),
                     "merge_tests": st["merge_tests"], "merge_distances": st["merge_distances"],
                     "merge_iterations": st["merge_iterations"]}
        log(f"bench: {name} {res[name]}")
    ctx.close()
    return res


def bench_learned(G, steps, warmup):
    """The dense seed-spreader workload (n=20M, d=3): the trained proposal
    versus the plain merge, same GPU, identical labels; beside it a 2M-point
    3-D sweep point at eps 2000 (619 core grids of about 3000 core points),
    where FastMerging's scans over large core sets dominate the merge."""
    w = W.WORKLOADS["cfg4"]
    res = learned_pair(G, points("cfg4"), w.eps, w.minpts, steps, warmup)
    out = {"workload": "seed-spreader n=20M d=3 eps=150 minpts=50 (300 pts/step)", "unit": "points/s",
           "value": res["learned"]["value"], "plain_value": res["plain"]["value"],
           "speedup_vs_plain": round(res["learned"]["value"] / res["plain"]["value"], 3),
           "plain": res["plain"], "learned": res["learned"]}
    import torch
    ws = W.sweep_workload("simden", 3, eps=2000)
    log(f"bench: generating {ws.name}")
    pts = torch.from_numpy(W.make_points(ws).astype(np.float32)).cuda()
    big = learned_pair(G, pts, ws.eps, ws.minpts, steps, warmup)
    out["large_core_sets"] = {
        "workload": "seed-spreader (simden) n=2M d=3 eps=2000 minpts=100, 817 grids",
        "speedup_vs_plain": round(big["learned"]["value"] / big["plain"]["value"], 3),
        "merge_speedup_vs_plain": round(big["plain"]["merge_ms"] / big["learned"]["merge_ms"], 3),
        "plain": big["plain"], "learned": big["learned"]}
    return out


def sweep_points(dims, kinds, axes):
    """(kind, d, n, eps, minpts) of every sweep point, each once, grouped by
    point set."""
    D = W.SWEEP_DEFAULT
    out = []
    for kind in kinds:
        for d in dims:
            pts = []
            if "eps" in axes:
                pts += [(D["n"], e, D["minpts"]) for e in W.SWEEP_EPS]
            if "minpts" in axes:
                pts += [(D["n"], D["eps"], m) for m in W.SWEEP_MINPTS]
            if "n" in axes:
                pts += [(n, D["eps"], D["minpts"]) for n in W.SWEEP_N]
            seen = set()
            for p in sorted(pts):
                if p not in seen:
                    seen.add(p)
                    out.append((kind, d) + p)
    return out


def bench_sweep(G, steps, warmup, dims, kinds, axes, path):
    """The paper's sweeps (Section 5.2): every point timed with the LDF order
    (GriT-DBSCAN-LDF) and with the breadth-first searches of Algorithm 6
    (GriT-DBSCAN); the two must give the same labels (Theorem 4), and where
    the oracle's digest of a point is stored the labels must equal it."""
    import hashlib
    import torch
    digests = (oracle_digest("sweep") or {})
    ctxs = {}
    for order, v in (("ldf", 1), ("bfs", 2)):
        ctxs[order] = G.Context(0)
        ctxs[order].set_option(G.GD_OPT_MERGE_ORDER, v)
    stat_ctx = G.Context(0)
    stat_ctx.set_option(G.GD_OPT_STATS, 1)
    cur_key, pts = None, None
    recs = []
    with open(path, "w") as f:
        for kind, d, n, eps, minpts in sweep_points(dims, kinds, axes):
            w = W.sweep_workload(kind, d, n, eps, minpts)
            if (kind, d, n) != cur_key:
                pts = None
                torch.cuda.empty_cache()
                log(f"sweep: generating {w.name}")
                pts = torch.from_numpy(W.make_points(w).astype(np.float32)).cuda()
                cur_key = (kind, d, n)
            lab = torch.empty(n, dtype=torch.int32, device="cuda")
            core = torch.empty(n, dtype=torch.uint8, device="cuda")
            rec = {"kind": kind, "d": d, "n": n, "eps": eps, "minpts": minpts}
            ref = None
            for order, ctx in ctxs.items():
                ms = []
                for i in range(warmup + steps):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    ctx.dbscan(pts, eps, minpts, lab, core)
                    if i >= warmup:
                        ms.append(1e3 * (time.perf_counter() - t0))
                rec[f"ms_{order}"] = round(float(np.median(ms)), 3)
                if ref is None:
                    ref = (lab.clone(), core.clone())
                elif not (torch.equal(ref[0], lab) and torch.equal(ref[1], core)):
                    raise RuntimeError(f"sweep {W.sweep_name(w)}: the BFS order changed the labels")
            rec["points_per_s_ldf"] = round(n / (rec["ms_ldf"] * 1e-3), 1)
            stat_ctx.dbscan(pts, eps, minpts, lab, core)
            st = stat_ctx.stats()
            l_np = ref[0].cpu().numpy()
            c_np = ref[1].cpu().numpy()
            rec.update({"key_bits": st["key_bits"], "grids": st["grids"], "core_grids": st["core_grids"],
                        "neighbor_entries": st["neighbor_entries"], "neighbor_walk": st["neighbor_walk"],
                        "merge_tests": st["merge_tests"], "merge_distances": st["merge_distances"],
                        "clusters": int(np.unique(l_np[l_np >= 0]).size), "core_points": int(c_np.sum()),
                        "noise_points": int((l_np < 0).sum())})
            dg = digests.get(W.sweep_name(w))
            if dg is not None:
                rec["labels_equal_oracle_digest"] = (
                    hashlib.sha256(np.ascontiguousarray(l_np.astype("<i4")).tobytes()).hexdigest() ==
                    dg["labels_sha256"] and
                    hashlib.sha256(np.ascontiguousarray(c_np.astype(np.uint8)).tobytes()).hexdigest() ==
                    dg["core_sha256"])
            f.write(json.dumps(rec) + "\n")
            f.flush()
            recs.append(rec)
            log(f"sweep: {W.sweep_name(w)} ldf {rec['ms_ldf']} ms bfs {rec['ms_bfs']} ms "
                f"clusters {rec['clusters']} bits {rec['key_bits']}")
    for ctx in list(ctxs.values()) + [stat_ctx]:
        ctx.close()
    return recs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="H", choices=sorted(W.WORKLOADS))
    ap.add_argument("--cpu-sample", type=int, default=3_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the batched and learned comparisons")
    ap.add_argument("--batch-instances", type=int, default=256)
    ap.add_argument("--neighbor-mode", type=int, default=0, choices=(0, 1, 2),
                    help="GD_OPT_NEIGHBOR_MODE: 0 auto, 1 lists for every grid, 2 walks in the consumers")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the 256-instance batched comparison and print its record")
    ap.add_argument("--sweep", metavar="FILE", help="run the parameter sweeps, one JSON record per point to FILE")
    ap.add_argument("--sweep-dims", default="2,3,5,7")
    ap.add_argument("--sweep-kinds", default="simden,varden")
    ap.add_argument("--sweep-axes", default="eps,minpts,n")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 512 MiB device copy (reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library clusters on one GPU (asked for --gpus {args.gpus}); "
              "sharding over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2210_07580_amd as G

    if args.batched_only:
        print(json.dumps({"batched": bench_batched(G, args.steps, args.warmup, args.batch_instances)}))
        return

    if args.sweep:
        recs = bench_sweep(G, args.steps, args.warmup, [int(v) for v in args.sweep_dims.split(",")],
                           args.sweep_kinds.split(","), args.sweep_axes.split(","), args.sweep)
        checked = [r["labels_equal_oracle_digest"] for r in recs if "labels_equal_oracle_digest" in r]
        print(json.dumps({"sweep_points": len(recs), "records": args.sweep, "steps": args.steps,
                          "warmup": args.warmup, "oracle_digests_checked": len(checked),
                          "oracle_digests_equal": sum(checked),
                          "total_ms_ldf": round(sum(r["ms_ldf"] for r in recs), 1),
                          "total_ms_bfs": round(sum(r["ms_bfs"] for r in recs), 1)}))
        return

    if args.copy_calibration:
        src = torch.ones(128 << 20, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("bench: copy calibration: 2 copies of 512 MiB")
        del src, dst

    w = W.WORKLOADS[args.workload]
    log(f"bench: generating {w.name} n={w.n:,} d={w.d}")
    x = W.make_points(w)
    n, d = x.shape
    dev = torch.device("cuda:0")
    pts = torch.from_numpy(x.astype(np.float32)).to(dev)
    labels = torch.empty(n, dtype=torch.int32, device=dev)
    core = torch.empty(n, dtype=torch.uint8, device=dev)
    ctx = G.Context(0)
    ctx.set_option(G.GD_OPT_NEIGHBOR_MODE, args.neighbor_mode)
    for i in range(args.warmup):
        ctx.dbscan(pts, w.eps, w.minpts, labels, core)
        log(f"bench: warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()

    step_ms = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        ctx.dbscan(pts, w.eps, w.minpts, labels, core)  # returns after the stream has drained
        step_ms.append(1e3 * (time.perf_counter() - ts))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"bench: {args.steps} timed steps done")
    # Phase durations: the same K steps again with a pair of HIP events
    # around every phase on the launch stream.  The events hold the stream
    # at each phase boundary (about 0.1 ms per call in all), so the steps
    # above run without them.
    ctx.set_option(G.GD_OPT_TIMING, 1)
    phase_sum = {}
    ti0 = time.perf_counter()
    for i in range(args.steps):
        ctx.dbscan(pts, w.eps, w.minpts, labels, core)
        for k, v in ctx.phase_times().items():
            phase_sum[k] = phase_sum.get(k, 0.0) + v
    torch.cuda.synchronize()
    t_instr = (time.perf_counter() - ti0) / args.steps
    ctx.set_option(G.GD_OPT_TIMING, 0)
    log(f"bench: {args.steps} steps with phase events done")
    # Work counters come from one more, untimed call with the device counters
    # on (the union order, hence the number of merge tests, varies slightly
    # from call to call).
    ctx.set_option(G.GD_OPT_STATS, 1)
    ctx.dbscan(pts, w.eps, w.minpts, labels, core)
    st = ctx.stats()
    ctx.set_option(G.GD_OPT_STATS, 0)
    # the same step replayed from a captured HIP graph (no host synchronisation between phases)
    ctx.set_option(G.GD_OPT_GRAPH, 2)
    t_graph = time_calls(lambda: ctx.dbscan(pts, w.eps, w.minpts, labels, core), args.steps, args.warmup)
    graph_ok = ctx.stats()["graph_replays"] == 1
    ctx.set_option(G.GD_OPT_GRAPH, 1)
    log(f"bench: graph replay {1e3 * t_graph:.3f} ms/step (replayed: {graph_ok})")

    K = args.steps
    total = t1 - t0
    ms_per_step = 1000.0 * total / K
    phases = {k: v / K for k, v in phase_sum.items()}
    packing = packed_rows(d, w.eps, st["key_bits"])
    key_bytes = 4 if st["key_bits"] <= 32 and packing != "word" else 8

    passes = (st["key_bits"] + 7) // 8
    traffic = measured_traffic(w.name)
    rooflines = {}
    for ph, ms in phases.items():
        b = algorithmic_bytes(ph, n, d, st, key_bytes, passes, packing)
        if b is None or ms <= 0:
            continue
        achieved = b / (ms * 1e-3) / 1e9
        t = traffic.get(ph)
        rooflines[ph] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": int(t["fetch_bytes"] + t["write_bytes"]) if t else None,
                         "avg_ms": round(ms, 4), "algorithmic_bytes": int(b)}
    dominant = max(rooflines, key=lambda k: rooflines[k]["avg_ms"])
    for ph in rooflines:
        rooflines[ph]["kernels"] = PHASE_KERNELS.get(ph, [])
    roofline = dict(kernel=dominant, **rooflines[dominant])

    out = {
        "metric": "points/sec exact DBSCAN (n=10M,d=3); batched & learned vs plain, same GPU",
        "value": round(n * K / total, 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "ms_min": round(min(step_ms), 3),
        "ms_median": round(float(np.median(step_ms)), 3),
        "ms_max": round(max(step_ms), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_DESC.get(w.name, w.name), "n": int(n), "d": int(d),
                   "eps": w.eps, "minpts": w.minpts, "seed": w.seed},
        "roofline": roofline,
        "rooflines": rooflines,
        "graph_replay": {"value": round(n / t_graph, 1), "ms_per_step": round(1e3 * t_graph, 3),
                         "replayed": graph_ok},
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "ms_per_step_with_phase_events": round(1e3 * t_instr, 3),
        "work": {k: st[k] for k in ("grids", "neighbor_entries", "core_points", "core_grids",
                                    "merge_pairs", "merge_skipped", "merge_tests", "merge_yes",
                                    "merge_max_iterations", "merge_distances", "merge_set_points", "core_distances",
                                    "core_candidates", "core_neighbor_grids", "key_bits")},
    }
    ctx.close()
    del pts, labels, core
    torch.cuda.empty_cache()
    if not args.no_variants:
        out["batched"] = bench_batched(G, max(2, args.steps // 2), 1, args.batch_instances)
        torch.cuda.empty_cache()
        out["learned"] = bench_learned(G, max(2, args.steps // 2), 1)
        few = max(3, min(args.steps, 10) // 2)
        out["configs"] = bench_configs(G, few, 1)
        out["merge_orders"] = bench_merge_orders(G, 3, 1)
        out["neighbor_modes"] = bench_neighbor_modes(G, 3, 1)
        out["approximate"] = bench_approx(G, 3, 1)
        _POINTS.clear()
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log(f"bench: CPU oracle on a sample of n={args.cpu_sample:,}")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
