#!/usr/bin/env python3
"""Train the learned-frontier predictor on traces of plain RAK runs.

Traces (lpa_trace) come from R-MAT graphs of scales 18-20 (seeds = scale,
edge factor 16, (a,b,c) = (0.57, 0.19, 0.19)) and two 1024 x 1024 damaged
lattices (seeds 1001 and 1002); R-MAT scale 20 with seed 120 is held out to
pick the decision threshold tau (the largest that still keeps `recall` of
the vertices that change).  Training (lpa_train) runs on the GPU with the
library's own forward, backward and Adam kernels.  The model is written as
JSON (weights as nested lists, the lpa_mlp field order).

    python -m paper_2301_09125_amd.train_frontier --out lf_model.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_MODEL = os.path.join(HERE, "lf_model.json")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def init_model(seed: int) -> dict:
    """He-initialised weights (float32 master copy)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return {"w1": (rng.standard_normal((6, 32)) * np.sqrt(2.0 / 6)).astype(np.float32),
            "b1": np.zeros(32, np.float32),
            "w2": (rng.standard_normal((32, 32)) * np.sqrt(2.0 / 32)).astype(np.float32),
            "b2": np.zeros(32, np.float32),
            "w3": (rng.standard_normal(32) * np.sqrt(1.0 / 32)).astype(np.float32),
            "b3": np.float32(0.0), "tau": 0.5}


def save_model(model: dict, path: str, meta: dict):
    out = {k: (v.tolist() if hasattr(v, "tolist") else v) for k, v in model.items()}
    out["b3"] = float(model["b3"])
    out["tau"] = float(model["tau"])
    out["meta"] = meta
    with open(path, "w") as f:
        json.dump(out, f)


def load_model(path: str = DEFAULT_MODEL) -> dict:
    import numpy as np
    d = json.load(open(path))
    m = {k: np.asarray(d[k], dtype=np.float32) for k in ("w1", "b1", "w2", "b2", "w3")}
    m["b3"] = np.float32(d["b3"])
    m["tau"] = float(d["tau"])
    return m


def training_graphs(gg, scales=(18, 19, 20), lattices=(1001, 1002)):
    for s in scales:
        yield f"rmat{s}", gg.rmat(s, 16, 0.57, 0.19, 0.19, seed=s)
    for seed in lattices:
        yield f"lattice1024_s{seed}", gg.road(1024, 1024, 0.3, 0.01, 0, 0, seed=seed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_MODEL)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=65536)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--recall", type=float, default=0.99)
    ap.add_argument("--tol", type=float, default=0.05)
    ap.add_argument("--max-iter", type=int, default=20)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--scales", type=int, nargs="*", default=[18, 19, 20])
    args = ap.parse_args()

    import torch
    import graphgen as gg
    import paper_2301_09125_amd as P

    ctx = P.Context(0)
    Xs, ys = [], []
    t0 = time.time()
    for name, g in training_graphs(gg, tuple(args.scales)):
        X, y = ctx.trace(P.DeviceGraph.from_csr(g, "cuda"), tol=args.tol, max_iter=args.max_iter)
        log(f"[train] trace {name}: n={g.n} m={g.m}: {X.shape[0]} samples, {int(y.sum())} changed")
        Xs.append(X)
        ys.append(y)
    X = torch.cat(Xs)
    y = torch.cat(ys)
    gv = gg.rmat(20, 16, 0.57, 0.19, 0.19, seed=120)
    Xv, yv = ctx.trace(P.DeviceGraph.from_csr(gv, "cuda"), tol=args.tol, max_iter=args.max_iter)
    pos = int(y.sum())
    pw = (X.shape[0] - pos) / max(pos, 1)
    log(f"[train] {X.shape[0]} samples ({pos} positive, pos_weight {pw:.3f}), validation {Xv.shape[0]}; "
        f"traces in {time.time() - t0:.1f}s")
    t1 = time.time()
    model, losses = ctx.train(X, y, init_model(args.seed), epochs=args.epochs, batch=args.batch, lr=args.lr,
                              pos_weight=pw, seed=args.seed, val=(Xv, yv), recall=args.recall)
    torch.cuda.synchronize()
    log(f"[train] losses {['%.4f' % x for x in losses]}, tau {model['tau']:.4f}, {time.time() - t1:.1f}s")
    meta = {"samples": int(X.shape[0]), "positives": pos, "pos_weight": pw, "epochs": args.epochs,
            "batch": args.batch, "lr": args.lr, "recall": args.recall, "losses": losses,
            "graphs": [f"rmat{s}" for s in args.scales] + ["lattice1024_s1001", "lattice1024_s1002"],
            "validation": "rmat20_s120"}
    save_model(model, args.out, meta)
    log(f"[train] wrote {args.out}")
    ctx.close()


if __name__ == "__main__":
    main()
