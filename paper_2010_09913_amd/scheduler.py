"""Learned per-level schedule: timing collection, training and evaluation.

Not in the paper.  Every variant of a level leaves bit-identical BFS state,
so the state a level sees does not depend on the variants chosen before it:
running a whole BFS with one forced variant times that variant on every level
of that BFS, and four such runs give the full per-level timing table.  The
features of a level are the same in all four runs.  Targets are the
log-times of the four variants centred per level and scaled by one deviation
(so the argmin is unchanged and only relative costs are learned); the MLP is
trained on the GPU by the library's own kernels (slimsell_sched_train).  The
saved model carries its training domain (the training features and a radius
tau), outside which the fixed heuristic decides.

Usage (writes the model next to this file):
  python -m paper_2010_09913_amd.scheduler --out paper_2010_09913_amd/models/sched_selmax.npy
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

from . import VARIANTS, Graph, sched_train

FORCED = ["pull", "pull-split256", "pull-split1024", "push"]
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_MODEL = os.path.join(HERE, "models", "sched_selmax.npy")


def collect(G: Graph, roots, semiring: str = "selmax", repeats: int = 3):
    """Per-level features and per-variant times (ms) for every root:
    returns (X [L, 6], T [L, 4])."""
    import torch
    xs, ts = [], []
    for root in roots:
        times, feats = [], None
        for mode in FORCED:
            G.bfs([int(root)], semiring, schedule=mode)  # warm
            reps = []
            for _ in range(repeats):
                res = G.bfs([int(root)], semiring, schedule=mode, level_cap=65536, timing=True,
                            counters=False)
                it = int(res.iterations[0])
                reps.append(res.levels["ms"][0][:it].copy())
            times.append(np.median(np.stack(reps), axis=0))
            if feats is None:
                feats = G.sched_log(it)[:, :6].copy()
        torch.cuda.synchronize()
        xs.append(feats)
        ts.append(np.stack(times, axis=1))
    return np.concatenate(xs), np.concatenate(ts)


def standardise(T):
    """Log-times centred per level (only the variants' relative cost is
    learned, which carries across graph sizes) and scaled by one deviation."""
    y = np.log(np.maximum(T, 1e-4))
    y = y - y.mean(axis=1, keepdims=True)
    sd = float(y.std() + 1e-6)
    return (y / sd).astype(np.float32), 0.0, sd


def train(X, T, steps: int = 3000, lr: float = 3e-3, seed: int = 0):
    y, mu, sd = standardise(T)
    w, losses = sched_train(X.astype(np.float32), y, steps=steps, lr=lr, seed=seed)
    return w, losses, (mu, sd)


def with_domain(w, X, quantile: float = 0.95, max_anchors: int = 1024):
    """The model with its training domain appended: the training features as
    anchors (an evenly spaced subset if there are more than max_anchors) and
    tau = the given quantile of each sample's distance to its nearest other
    sample, so a level the training data does not cover is left to the
    heuristic."""
    X = np.asarray(X, np.float64)
    if len(X) > max_anchors:
        X = X[np.linspace(0, len(X) - 1, max_anchors).astype(np.int64)]
    d = np.sqrt(((X[:, None, :] - X[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(d, np.inf)
    tau = float(np.quantile(d.min(1), quantile)) if len(X) > 1 else 0.1
    tau = max(tau, 1e-3)
    return np.concatenate([np.asarray(w, np.float32).ravel(),
                           np.array([tau, len(X)], np.float32),
                           X.astype(np.float32).ravel()]), tau


def evaluate(G: Graph, roots, semiring: str = "selmax", modes=None):
    """Total BFS time (ms, events) over the roots for each schedule."""
    import torch
    modes = modes or ["learned", "heuristic", *FORCED]
    out = {}
    for mode in modes:
        G.bfs([int(roots[0])], semiring, schedule=mode)  # warm
        total = 0.0
        for root in roots:
            res = G.bfs([int(root)], semiring, schedule=mode, timing="bfs")
            total += float(res.runs["bfs_ms"][0])
        torch.cuda.synchronize()
        out[mode] = total
    return out


def training_graphs():
    """The graphs of configurations 1-3 with their roots."""
    import graphgen
    yield "rmat-s12", graphgen.rmat(12, 16, seed=1), None
    e = graphgen.rmat(20, 16, seed=1)
    yield "rmat-s20", e, graphgen.pick_roots(e, 16, seed=1001)
    e = graphgen.rmat(22, 16, seed=1)
    yield "rmat-s22", e, graphgen.pick_roots(e, 64, seed=1002)
    e = graphgen.er(1 << 22, 16 << 22, seed=2)
    yield "er-2^22", e, graphgen.pick_roots(e, 64, seed=1003)


def main() -> int:
    ap = argparse.ArgumentParser(description="train the per-level scheduler on this GPU")
    ap.add_argument("--out", default=DEFAULT_MODEL)
    ap.add_argument("--roots", type=int, default=16, help="roots per graph")
    ap.add_argument("--repeats", type=int, default=3)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--semiring", default="selmax")
    args = ap.parse_args()
    import torch
    Xs, Ts, meta = [], [], []
    for name, e, roots in training_graphs():
        t = time.perf_counter()
        G = Graph.from_edgelist(e, sigma=0)
        if roots is None:
            deg = G.degrees()
            roots = np.array([int(np.argmax(deg))], np.int32)
        roots = roots[: args.roots]
        X, T = collect(G, roots, args.semiring, args.repeats)
        G.close()
        torch.cuda.synchronize()
        Xs.append(X)
        Ts.append(T)
        meta.append({"graph": name, "roots": int(len(roots)), "levels": int(len(X))})
        print(f"{name}: {len(X)} levels in {time.perf_counter() - t:.1f}s; best variant counts "
              f"{np.bincount(np.argmin(T, 1), minlength=4).tolist()}", flush=True)
    X, T = np.concatenate(Xs), np.concatenate(Ts)
    w, losses, (mu, sd) = train(X, T, steps=args.steps)
    from . import sched_forward
    pred = np.argmin(sched_forward(w, X), 1)
    best_possible = T.min(1).sum()
    chosen = T[np.arange(len(T)), pred].sum()
    print(json.dumps({"samples": int(len(X)), "loss_first": float(losses[0]),
                      "loss_last": float(losses[-1]), "chosen_ms": float(chosen),
                      "best_possible_ms": float(best_possible),
                      "forced_ms": {v: float(T[:, i].sum()) for i, v in enumerate(VARIANTS)},
                      "graphs": meta}), flush=True)
    model, tau = with_domain(w, X)
    print(json.dumps({"domain_tau": tau, "anchors": int(min(len(X), 1024))}), flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, model)
    np.save(os.path.splitext(args.out)[0] + "_data.npy",
            np.concatenate([X, T], axis=1).astype(np.float32))
    return 0


if __name__ == "__main__":
    sys.exit(main())
