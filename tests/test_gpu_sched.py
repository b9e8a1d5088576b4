"""GPU tests of the learned per-level schedule: MLP kernels against the
float64 oracle, training, and exact BFS results under every schedule."""
import sys

import numpy as np
import pytest

import graphgen
import oracle
from oracle import mlp

pytestmark = pytest.mark.gpu
SEMIS = ["tropical", "real", "boolean", "selmax"]


@pytest.fixture(scope="module")
def ss():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2010_09913_amd as mod
    return mod


def note(*a):
    print(*a, file=sys.stderr, flush=True)


def test_gradient_and_forward_match_the_oracle(ss):
    rng = np.random.default_rng(1)
    w = rng.normal(0, 0.3, mlp.PARAMS).astype(np.float32)
    x = rng.random((777, 6)).astype(np.float32)
    y = rng.normal(0, 1, (777, 4)).astype(np.float32)
    loss, g = ss.sched_grad(w, x, y)
    ref_loss, ref_g = mlp.loss_and_grad(w.astype(np.float64), x.astype(np.float64),
                                        y.astype(np.float64))
    assert abs(loss - ref_loss) <= 1e-5 * abs(ref_loss)
    np.testing.assert_allclose(g, ref_g, rtol=1e-4, atol=1e-4 * np.abs(ref_g).max())
    out = ss.sched_forward(w, x)
    np.testing.assert_allclose(out, mlp.forward(w, x), rtol=1e-5, atol=1e-5)


def test_training_reduces_loss_and_is_deterministic(ss):
    rng = np.random.default_rng(2)
    teacher = rng.normal(0, 0.5, mlp.PARAMS)
    x = rng.random((1500, 6)).astype(np.float32)
    y = mlp.forward(teacher, x).astype(np.float32)
    w1, l1 = ss.sched_train(x, y, steps=600, lr=3e-3, seed=7)
    w2, l2 = ss.sched_train(x, y, steps=600, lr=3e-3, seed=7)
    np.testing.assert_array_equal(w1, w2)
    assert l1[-1] < 0.1 * l1[0]
    assert abs(mlp.loss_only(w1, x, y) - l1[-1]) < 0.05 * l1[-1] + 1e-6


def _graphs():
    return {
        "rmat": graphgen.rmat(13, 16, seed=41),
        "er": graphgen.er(6000, 30000, seed=42),
        "grid": graphgen.grid(64, 48, 0.05, seed=5),
        "path": graphgen.EdgeList(300, np.arange(299, dtype=np.int32),
                                  np.arange(1, 300, dtype=np.int32), "path300"),
    }


def _run(G, root, semi, schedule, persistent=False):
    import torch
    res = G.bfs([root], semi, schedule=schedule, level_cap=4096, persistent=persistent)
    torch.cuda.synchronize()
    return res


def _check(res, ex, semi):
    np.testing.assert_array_equal(res.dist[0].cpu().numpy(), ex.dist)
    assert int(res.iterations[0]) == ex.iterations
    if semi == "selmax":
        np.testing.assert_array_equal(res.parent[0].cpu().numpy(), ex.parent)
    if semi == "real":
        np.testing.assert_array_equal(res.real_val[0].cpu().numpy(), ex.real_val)


@pytest.mark.parametrize("name", ["rmat", "er", "grid", "path"])
def test_every_schedule_is_exact_and_features_match(ss, name):
    e = _graphs()[name]
    g = oracle.csr_from_edgelist(e)
    G = ss.Graph.from_edgelist(e)
    roots = graphgen.pick_roots(e, 2, seed=43)
    rng = np.random.default_rng(3)
    random_model = rng.normal(0, 0.5, mlp.PARAMS).astype(np.float32)
    pull_v = 1  # the default split length (at most 512) maps to the split-256 pull variant
    for root in roots:
        ex = oracle.expected(g, int(root))
        feats = mlp.features(ex.dist, g.degree, g.n, g.entries)
        heur = mlp.heuristic(ex.dist, g.degree, g.n, g.entries, pull_v)
        for semi in SEMIS:
            for mode in ["heuristic", "pull", "pull-split256", "pull-split1024", "push"]:
                note(name, root, semi, mode)
                res = _run(G, int(root), semi, mode)
                _check(res, ex, semi)
                it = ex.iterations
                var = res.levels["variant"][0][:it]
                if mode == "heuristic":
                    log = G.sched_log(it)
                    np.testing.assert_allclose(log[:, :6], feats, rtol=0, atol=2e-6)
                    np.testing.assert_array_equal(log[:, 11], np.arange(1, it + 1))
                    # compare the decisions away from ties of the float32 rule
                    np.testing.assert_array_equal(var, heur)
                else:
                    assert np.all(var == ss.VARIANTS.index(mode))
                # one cooperative launch: same results, same decisions
                note(name, root, semi, mode, "persistent")
                resp = _run(G, int(root), semi, mode, persistent=True)
                _check(resp, ex, semi)
                assert int(resp.runs["launches"][0]) == 1
                np.testing.assert_array_equal(resp.levels["variant"][0][:it], var)
            # learned: random model -> exact; scores equal the oracle's forward
            ss.sched_load(random_model)
            resp = _run(G, int(root), semi, "learned", persistent=True)
            _check(resp, ex, semi)
            logp = G.sched_log(ex.iterations)
            res = _run(G, int(root), semi, "learned")
            _check(res, ex, semi)
            log = G.sched_log(ex.iterations)
            np.testing.assert_array_equal(logp, log)
            ref = mlp.forward(random_model, log[:, :6])
            np.testing.assert_allclose(log[:, 6:10], ref, rtol=1e-5, atol=1e-5)
            srt = np.sort(ref, axis=1)
            clear = (srt[:, 1] - srt[:, 0]) > 1e-3
            np.testing.assert_array_equal(log[clear, 10], np.argmin(ref, axis=1)[clear])
            ss.sched_clear()
    G.close()


def test_model_that_prefers_one_variant_and_nan_fallback(ss):
    e = _graphs()["rmat"]
    g = oracle.csr_from_edgelist(e)
    G = ss.Graph.from_edgelist(e)
    root = int(graphgen.pick_roots(e, 1, seed=44)[0])
    ex = oracle.expected(g, root)
    for v in range(4):
        w = np.zeros(mlp.PARAMS, np.float32)
        w[-4:] = 1.0
        w[-4 + v] = -1.0                    # b3: variant v always scores lowest
        ss.sched_load(w)
        res = _run(G, root, "selmax", "learned")
        _check(res, ex, "selmax")
        assert np.all(res.levels["variant"][0][:ex.iterations] == v)
    w = np.full(mlp.PARAMS, np.nan, np.float32)
    ss.sched_load(w)
    res = _run(G, root, "selmax", "learned")
    _check(res, ex, "selmax")
    heur = _run(G, root, "selmax", "heuristic")
    np.testing.assert_array_equal(res.levels["variant"][0], heur.levels["variant"][0])
    ss.sched_clear()
    res = _run(G, root, "selmax", "learned")   # no model: heuristic
    np.testing.assert_array_equal(res.levels["variant"][0], heur.levels["variant"][0])
    # whole-BFS timing only: no per-level events
    for pers in (False, True):
        rt = G.bfs([root], "selmax", schedule="heuristic", timing="bfs", persistent=pers)
        _check(rt, ex, "selmax")
        assert rt.runs["bfs_ms"][0] > 0 and rt.runs["kernel_ms"][0] == 0
    with pytest.raises(ss.SlimSellError):
        G.bfs([root], "selmax", schedule="heuristic", slimwork=1)
    with pytest.raises(ss.SlimSellError):
        ss.sched_load(np.zeros(10, np.float32))
    G.close()


def _offsets(rng, shape, length):
    d = rng.normal(size=shape)
    return (length * d / np.linalg.norm(d, axis=1, keepdims=True)).astype(np.float32)


def test_training_domain_decides_between_model_and_heuristic(ss):
    e = _graphs()["rmat"]
    g = oracle.csr_from_edgelist(e)
    G = ss.Graph.from_edgelist(e)
    rng = np.random.default_rng(5)
    w = rng.normal(0, 0.5, mlp.PARAMS).astype(np.float32)
    for root in graphgen.pick_roots(e, 2, seed=46):
        ex = oracle.expected(g, int(root))
        it = ex.iterations
        feats = mlp.features(ex.dist, g.degree, g.n, g.entries).astype(np.float32)
        heur = mlp.heuristic(ex.dist, g.degree, g.n, g.entries, 1)
        cases = {
            # every level on an anchor: the model decides everywhere
            "inside": (feats, 1e-3),
            # anchors far from every level: the heuristic decides everywhere
            "outside": (feats + 5.0, 0.5),
            # every other level is an anchor, tau below the gaps: mixed
            "mixed": (feats[::2], 1e-3),
            # every level half of tau from its anchor in a random direction:
            # inside, though level and anchor may sit in different cells of
            # the domain box's map, which must not clear the level's cell
            "near": (feats + _offsets(rng, feats.shape, 0.5 * 0.05), 0.05),
        }
        for name, (anchors, tau) in cases.items():
            note("domain", root, name)
            model = np.concatenate([w, [tau, len(anchors)], anchors.ravel()]).astype(np.float32)
            ss.sched_load(model)
            res = _run(G, int(root), "selmax", "learned")
            _check(res, ex, "selmax")
            got = res.levels["variant"][0][:it]
            want, scores = mlp.choose(model, feats, heur)
            # compare away from ties of the scores and of the distance test
            srt = np.sort(scores, axis=1)
            d2 = mlp.nearest_anchor_sq(feats, anchors)
            clear = ((srt[:, 1] - srt[:, 0]) > 1e-3) & (np.abs(d2 - np.float32(tau) ** 2) > 1e-6)
            np.testing.assert_array_equal(got[clear], want[clear])
            if name == "outside":
                np.testing.assert_array_equal(got, heur)
            # the persistent form decides the same
            resp = _run(G, int(root), "selmax", "learned", persistent=True)
            _check(resp, ex, "selmax")
            np.testing.assert_array_equal(resp.levels["variant"][0][:it], got)
    for bad in ([0.0, 1.0], [0.1, 0.0], [0.1, 2.0], [np.nan, 1.0]):
        with pytest.raises(ss.SlimSellError):
            ss.sched_load(np.concatenate([w, bad, np.zeros(6)]).astype(np.float32))
    ss.sched_clear()
    G.close()


def test_model_staged_inside_the_box_decides_the_same(ss):
    """The learned schedule decides identically whether the model is staged
    before the domain test (a graph's first learned run, or after a run with
    some level inside the domain) or only for levels inside the domain
    (forced, or by itself after a run with none): same outputs and the same
    log (features, scores, variants) bit for bit, per-level and persistent."""
    e = _graphs()["rmat"]
    g = oracle.csr_from_edgelist(e)
    G = ss.Graph.from_edgelist(e)
    rng = np.random.default_rng(7)
    w = rng.normal(0, 0.5, mlp.PARAMS).astype(np.float32)
    root = int(graphgen.pick_roots(e, 1, seed=47)[0])
    ex = oracle.expected(g, root)
    it = ex.iterations
    feats = mlp.features(ex.dist, g.degree, g.n, g.entries).astype(np.float32)

    def run(model, **kw):
        import torch
        ss.sched_load(model)
        res = G.bfs([root], "selmax", schedule="learned", level_cap=4096, **kw)
        torch.cuda.synchronize()
        _check(res, ex, "selmax")
        return res.levels["variant"][0][:it].copy(), G.sched_log(it)

    try:
        for name, anchors, tau in (("inside", feats, 1e-3), ("mixed", feats[::2], 1e-3),
                                   ("outside", feats + 5.0, 0.5)):
            note("staging", name)
            model = np.concatenate([w, [tau, len(anchors)], anchors.ravel()]).astype(np.float32)
            v_eager, log_eager = run(model)                   # up front (default)
            v_lazy, log_lazy = run(model, sched_lazy=True)    # only inside the box
            np.testing.assert_array_equal(v_lazy, v_eager)
            np.testing.assert_array_equal(log_lazy, log_eager)
            # after the forced run the graph chooses by itself again; the
            # persistent form decides the same as well
            v_auto, log_auto = run(model)
            np.testing.assert_array_equal(v_auto, v_eager)
            np.testing.assert_array_equal(log_auto, log_eager)
            v_p, _ = run(model, persistent=True, sched_lazy=True)
            np.testing.assert_array_equal(v_p, v_eager)
    finally:
        ss.sched_clear()
        G.close()
