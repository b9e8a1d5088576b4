"""ORACLE -- test infrastructure only.

Float64 reference of the per-level scheduler: its six frontier features (from
BFS distances and degrees, by their definitions) and the MLP 6 -> 32 -> 32 -> 4
(ReLU) with its mean-squared-error loss and gradient written out by hand.
The scheduler is not in the paper; its definitions are the ones stated in
include/slimsell.h.  Pinned by central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np

H, F, V = 32, 6, 4
SIZES = [("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (V, H)), ("b3", (V,))]
PARAMS = sum(int(np.prod(s)) for _, s in SIZES)  # 1412


def unpack(w):
    w = np.asarray(w, np.float64).reshape(-1)
    assert w.shape[0] == PARAMS
    out, off = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = w[off:off + k].reshape(shape)
        off += k
    return out


def forward(w, x):
    p = unpack(w)
    x = np.asarray(x, np.float64).reshape(-1, F)
    a1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    return h2 @ p["W3"].T + p["b3"]


def loss_and_grad(w, x, y):
    """L = mean over all N x 4 outputs of (out - y)^2 and dL/dw (flat)."""
    p = unpack(w)
    x = np.asarray(x, np.float64).reshape(-1, F)
    y = np.asarray(y, np.float64).reshape(-1, V)
    n = x.shape[0]
    a1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    out = h2 @ p["W3"].T + p["b3"]
    e = out - y
    loss = float(np.sum(e * e) / (n * V))
    d_out = 2.0 * e / (n * V)
    gW3 = d_out.T @ h2
    gb3 = d_out.sum(0)
    d_h2 = (d_out @ p["W3"]) * (a2 > 0)
    gW2 = d_h2.T @ h1
    gb2 = d_h2.sum(0)
    d_h1 = (d_h2 @ p["W2"]) * (a1 > 0)
    gW1 = d_h1.T @ x
    gb1 = d_h1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def loss_only(w, x, y):
    out = forward(w, x)
    y = np.asarray(y, np.float64).reshape(-1, V)
    return float(np.mean((out - y) ** 2))


def features(dist, degree, n: int, entries: int):
    """Features of levels 1..D+1 of one BFS: row k-1 describes level k.
    n_f, m_f: vertices and degree sum at distance k-1; m_u: degree sum at
    distance >= k or unreachable.  The frontier's size (vertices, edges) and
    the unvisited edges relative to the graph, the frontier's mean degree, the
    unvisited edges per vertex of the graph, and the frontier/unvisited edge
    ratio, all on log scales."""
    dist = np.asarray(dist)
    deg = np.asarray(degree, np.float64)
    iters = int(dist.max()) + 1
    l2n = np.log2(max(n, 2.0))
    l2m = np.log2(1.0 + max(float(entries), 1.0))
    rows = []
    for k in range(1, iters + 1):
        at = dist == k - 1
        before = (dist >= 0) & (dist < k)
        nf = float(at.sum())
        mf = float(deg[at].sum())
        mu = max(float(entries - deg[before].sum()), 0.0)
        fdeg = np.clip(np.log2((1.0 + mf) / (1.0 + nf)) / 16.0, 0.0, 1.0)
        udeg = np.clip(np.log2((1.0 + mu) / n) / 8.0, -1.0, 1.0)
        ratio = np.clip(np.log2((1.0 + mf) / (1.0 + mu)) / 16.0, -1.0, 1.0)
        rows.append([np.log2(1.0 + nf) / l2n, np.log2(1.0 + mf) / l2m, np.log2(1.0 + mu) / l2m,
                     fdeg, udeg, ratio])
    return np.array(rows)


def heuristic(dist, degree, n: int, entries: int, pull_variant: int):
    """The fixed fallback rule per level: the pull variant once
    m_f * 14 > m_u, otherwise push (3)."""
    dist = np.asarray(dist)
    deg = np.asarray(degree, np.float64)
    out = []
    for k in range(1, int(dist.max()) + 2):
        at = dist == k - 1
        before = (dist >= 0) & (dist < k)
        nf, mf = float(at.sum()), float(deg[at].sum())
        nu, mu = float(n - before.sum()), float(entries - deg[before].sum())
        pull = mf * 14.0 > mu
        out.append(pull_variant if pull else 3)
    return np.array(out)


def split_domain(model):
    """A model is the 1412 MLP parameters, optionally followed by its training
    domain: tau, K and K feature vectors.  Returns (params, tau, anchors)."""
    model = np.asarray(model, np.float64)
    w = model[:PARAMS]
    if model.size == PARAMS:
        return w, None, None
    tau, k = float(model[PARAMS]), int(model[PARAMS + 1])
    return w, tau, model[PARAMS + 2: PARAMS + 2 + 6 * k].reshape(k, 6)


def nearest_anchor_sq(x, anchors):
    """Squared distance from each feature row to its nearest anchor, in float32
    (the precision the schedule decides in)."""
    x = np.asarray(x, np.float32)
    a = np.asarray(anchors, np.float32)
    d = x[:, None, :] - a[None, :, :]
    return (d * d).sum(-1, dtype=np.float32).min(1)


def choose(model, x, heuristic_variants):
    """The learned schedule's decision per level: the variant of smallest
    predicted log-time when the level lies within tau of a training anchor
    (or the model carries no domain) and the scores are finite, otherwise
    the heuristic's variant."""
    w, tau, anchors = split_domain(model)
    scores = forward(w, x)
    pick = np.argmin(scores, axis=1)
    ok = np.all(np.isfinite(scores), axis=1)
    if anchors is not None:
        ok &= nearest_anchor_sq(x, anchors) <= np.float32(tau) * np.float32(tau)
    return np.where(ok, pick, np.asarray(heuristic_variants)), scores
