"""Pins of the float64 scheduler oracle: central finite differences for the
gradient, a hand-computed forward pass, and hand-computed features."""
import numpy as np

import graphgen
import oracle
from oracle import mlp


def test_gradient_matches_central_finite_differences():
    rng = np.random.default_rng(0)
    w = rng.normal(0, 0.4, mlp.PARAMS)
    x = rng.random((37, 6))
    y = rng.normal(0, 1, (37, 4))
    loss, g = mlp.loss_and_grad(w, x, y)
    assert abs(loss - mlp.loss_only(w, x, y)) < 1e-12
    h = 1e-6
    idx = rng.choice(mlp.PARAMS, 300, replace=False)
    fd = np.array([(mlp.loss_only(w + h * np.eye(1, mlp.PARAMS, i)[0], x, y)
                    - mlp.loss_only(w - h * np.eye(1, mlp.PARAMS, i)[0], x, y)) / (2 * h)
                   for i in idx])
    np.testing.assert_allclose(g[idx], fd, rtol=1e-6, atol=1e-9)


def test_forward_by_hand():
    w = np.zeros(mlp.PARAMS)
    p = mlp.unpack(w)            # views into w
    p["W1"][0, 2] = 2.0          # h1_0 = relu(2 x_2 - 1)
    p["b1"][0] = -1.0
    p["W2"][5, 0] = 3.0          # h2_5 = relu(3 h1_0)
    p["W3"][1, 5] = -0.5         # out_1 = -0.5 h2_5 + 7
    p["b3"][1] = 7.0
    x = np.array([[0, 0, 2.0, 0, 0, 0], [0, 0, 0.25, 0, 0, 0]])
    out = mlp.forward(w, x)
    np.testing.assert_allclose(out, [[0, 7 - 0.5 * 9, 0, 0], [0, 7, 0, 0]])


def test_features_by_hand_on_a_star():
    # star with centre 0 and 9 leaves; root = centre; m = 9 edges, 2m = 18
    e = graphgen.EdgeList(10, np.zeros(9, np.int32), np.arange(1, 10, dtype=np.int32), "star")
    g = oracle.csr_from_edgelist(e)
    d = oracle.bfs(g, 0)
    f = mlp.features(d, g.degree, 10, g.entries)
    l2n, l2m = np.log2(10), np.log2(19)
    # level 1: frontier {0} (deg 9); unvisited: 9 leaves, 9 edge ends
    np.testing.assert_allclose(f[0], [np.log2(2) / l2n, np.log2(10) / l2m, np.log2(10) / l2m,
                                      0.9, np.log2(2) / 8, 0.0])
    # level 2: frontier = 9 leaves (deg 1 each); nothing unvisited
    np.testing.assert_allclose(f[1], [np.log2(10) / l2n, np.log2(10) / l2m, 0.0, 0.0,
                                      np.log2(10 / 2) / 8, np.log2(10) / 16])
    assert len(f) == 2
    h = mlp.heuristic(d, g.degree, 10, g.entries, pull_variant=1)
    assert h.tolist() == [1, 1]   # 9*14 > 9: pull; then 9*14 > 0: pull
