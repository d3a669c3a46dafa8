"""Write SHA-256 digests of the CPU oracle's full-size results.

Runs the seeded generators and the oracle only (never the GPU library) and
stores, per workload, the digest of the generated points (so a changed
generator is told apart from a wrong result), the digests of the oracle's
int32 labels and uint8 core flags, and a few counts for diagnosis.

    python tests/golden/make_oracle_digests.py cfg1 H cfg4 cfg2 [--threads N]
    python tests/golden/make_oracle_digests.py cfg3 [--threads N]
    python tests/golden/make_oracle_digests.py ss-varden-7d/n=2000000/eps=500/minpts=100 ...

``cfg3`` is the 256-instance batch workload: one record per instance, in
instance order, under the key "cfg3".  Names of the form
``ss-<kind>-<d>d/n=../eps=../minpts=..`` are points of the parameter sweeps,
stored under the key "sweep".
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_digests.json")


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def record(w, x, labels, core, seconds, threads):
    return {
        "n": int(x.shape[0]), "d": int(x.shape[1]), "eps": w.eps, "minpts": w.minpts,
        "points_sha256": digest(x),
        "labels_sha256": digest(labels.astype("<i4")),
        "core_sha256": digest(core.astype(np.uint8)),
        "clusters": int(np.unique(labels[labels >= 0]).size),
        "core_points": int(core.sum()),
        "noise_points": int((labels < 0).sum()),
        "oracle_seconds": round(seconds, 1),
        "oracle_threads": threads,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+")
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    db = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            db = json.load(f)
    threads = args.threads or oracle.max_threads()
    for name in args.names:
        if name == "cfg3":
            recs = []
            for k, w in enumerate(W.batch_workloads()):
                x = W.make_points(w)
                t0 = time.time()
                labels, core = oracle.dbscan(x, w.eps, w.minpts, nthreads=threads)
                recs.append(record(w, x, labels, core, time.time() - t0, threads))
                print(f"cfg3 instance {k}: n={x.shape[0]} d={x.shape[1]} {recs[-1]['oracle_seconds']} s", flush=True)
            db[name] = recs
            with open(OUT, "w") as f:
                json.dump(db, f, indent=1, sort_keys=True)
            continue
        sweep = name.startswith("ss-")
        w = W.sweep_from_name(name) if sweep else W.WORKLOADS[name]
        x = W.make_points(w)
        t0 = time.time()
        labels, core = oracle.dbscan(x, w.eps, w.minpts, nthreads=threads)
        dt = time.time() - t0
        rec = record(w, x, labels, core, dt, threads)
        if sweep:
            db.setdefault("sweep", {})[W.sweep_name(w)] = rec
        else:
            db[name] = rec
        print(name, json.dumps(rec), flush=True)
        with open(OUT, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
