"""Train the learned proposal on the GPU and write proposal_fp16.bin.

Training pairs come from the method's own merges on the seed-spreader (n=2M,
d=3) and Gaussian-blob (d=5) workloads; training and inference use the
library's FP16 kernels.

    python -m paper_2210_07580_amd.train_proposal [--out PATH] [--steps N]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    import torch

    import workloads as W
    from paper_2210_07580_amd import Context
    from paper_2210_07580_amd import proposal as P

    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=P.BLOB_PATH)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--samples", type=int, default=120_000)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()

    ctx = Context(0)
    sets = [("cfg1", None), ("cfg2", 2_000_000)]
    Xs, Ts, Cs = [], [], []
    for name, n in sets:
        w = W.WORKLOADS[name]
        x = W.make_points(w, n=n)
        pts = torch.from_numpy(x.astype(np.float32)).cuda()
        X, T, C = P.harvest_from(ctx, pts, w.eps, w.minpts, args.samples, seed=args.seed)
        print(f"harvest {name} n={len(x)}: {X.shape[0]} pairs, merged {float(T[:, 0].mean()):.3f}, "
              f"b-side cheaper {float(T[:, 1].mean()):.3f}", flush=True)
        Xs.append(X)
        Ts.append(T)
        Cs.append(C)
    X = torch.cat(Xs)
    T = torch.cat(Ts)
    # hold out 10% to report accuracy
    S = X.shape[0]
    perm = torch.from_numpy(np.random.default_rng(args.seed).permutation(S)).cuda()
    cut = S // 10
    Xv, Tv = X[perm[:cut]].contiguous(), T[perm[:cut]].contiguous()
    Xt, Tt = X[perm[cut:]].contiguous(), T[perm[cut:]].contiguous()
    blob, losses = P.train(ctx, Xt, Tt, steps=args.steps, seed=args.seed)
    Z = ctx.mlp_forward(Xv, torch.from_numpy(blob).cuda()).cpu().numpy()
    tv = Tv.cpu().numpy()
    acc0 = float(((Z[:, 0] > 0) == (tv[:, 0] > 0.5)).mean())
    m = tv[:, 2] > 0.5
    acc1 = float(((Z[m, 1] > 0) == (tv[m, 1] > 0.5)).mean()) if m.any() else float("nan")
    P.save_blob(blob, args.out)
    print(json.dumps({"samples": int(S), "steps": args.steps, "loss_first": float(losses[:50].mean()),
                      "loss_last": float(losses[-50:].mean()), "heldout_merge_accuracy": acc0,
                      "heldout_side_accuracy": acc1, "out": args.out}), flush=True)


if __name__ == "__main__":
    main()
