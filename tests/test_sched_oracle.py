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
    # (n_f = 1, m_f = 9, m_u = 9: mean frontier degree log2(10/2)/16, unvisited
    # edge ends per vertex log2(10/10)/8 = 0, ratio 0)
    np.testing.assert_allclose(f[0], [np.log2(2) / l2n, np.log2(10) / l2m, np.log2(10) / l2m,
                                      np.log2(5) / 16, 0.0, 0.0])
    # level 2: frontier = 9 leaves (deg 1 each); nothing unvisited
    # (m_u = 0: log2(1/10)/8 for the unvisited edge ends per vertex)
    np.testing.assert_allclose(f[1], [np.log2(10) / l2n, np.log2(10) / l2m, 0.0,
                                      0.0, np.log2(0.1) / 8, np.log2(10) / 16])
    assert len(f) == 2
    h = mlp.heuristic(d, g.degree, 10, g.entries, pull_variant=1)
    assert h.tolist() == [1, 1]   # 9*14 > 9: pull; then 9*14 > 0: pull


def test_domain_rule_by_hand():
    """A level inside tau of an anchor follows the model, one outside falls
    back to the heuristic; a model without a domain always answers."""
    w = np.zeros(mlp.PARAMS)
    w[-4:] = [1.0, 2.0, 3.0, 0.0]          # b3: variant 3 always scores lowest
    anchors = np.array([[0.1, 0.2, 0.3, 0.4, 0.5, 0.6]])
    model = np.concatenate([w, [0.1, 1.0], anchors.ravel()])
    x = np.array([[0.1, 0.2, 0.3, 0.4, 0.5, 0.6],       # on the anchor
                  [0.1, 0.2, 0.3, 0.4, 0.5, 0.69],      # 0.09 away: inside
                  [0.1, 0.2, 0.3, 0.4, 0.5, 0.75]])     # 0.15 away: outside
    pick, _ = mlp.choose(model, x, [1, 1, 1])
    assert pick.tolist() == [3, 3, 1]
    pick, _ = mlp.choose(w, x, [1, 1, 1])
    assert pick.tolist() == [3, 3, 3]
    p, tau, a = mlp.split_domain(model)
    assert tau == 0.1 and a.shape == (1, 6) and p.size == mlp.PARAMS
