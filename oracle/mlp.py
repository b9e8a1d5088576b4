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
    n_f, m_f: vertices and degree sum at distance k-1; n_u, m_u: vertices and
    degree sum at distance >= k or unreachable; prev: vertices at k-2."""
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
        nu = float(n - before.sum())
        mu = float(entries - deg[before].sum())
        prev = float((dist == k - 2).sum()) if k >= 2 else 0.0
        growth = np.clip(np.log2((1.0 + nf) / (1.0 + prev)) / 8.0, -1.0, 1.0)
        ratio = np.clip(np.log2((1.0 + mf) / (1.0 + max(mu, 0.0))) / 16.0, -1.0, 1.0)
        rows.append([np.log2(1.0 + nf) / l2n, np.log2(1.0 + mf) / l2m,
                     np.log2(1.0 + max(mu, 0.0)) / l2m, max(nu, 0.0) / n, growth, ratio])
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
