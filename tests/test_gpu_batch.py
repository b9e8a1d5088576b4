"""GPU parity of the batched boolean SpMM (64-bit frontier masks), of
multi-graph unions, and of the autotuner, against the CPU oracle."""
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ss():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2010_09913_amd as mod
    return mod


def note(*a):
    print(*a, file=sys.stderr, flush=True)


def _check_batch(G, graphs, csrs, roots, slots_to_check=None, **kw):
    """roots [num_graphs, rpg]; compare every (graph, slot) or a sample."""
    import torch
    dist, iters, levels, runs = G.bfs_batch(roots, **kw)
    torch.cuda.synchronize()
    d = dist.cpu().numpy()
    ns, off = G.parts()
    rpg = roots.shape[1]
    max_ecc = 0
    for i, (g, c) in enumerate(zip(graphs, csrs)):
        blk = d[rpg * off[i]: rpg * (off[i] + ns[i])].reshape(rpg, ns[i])
        slots = range(rpg) if slots_to_check is None else slots_to_check
        for b in slots:
            r = int(roots[i, b])
            if r < 0:
                assert np.all(blk[b] == -1)
                continue
            ex = oracle.bfs(c, r)
            np.testing.assert_array_equal(blk[b], ex, err_msg=f"graph {i} slot {b} root {r} {kw}")
            max_ecc = max(max_ecc, int(ex.max()))
    if slots_to_check is None:
        assert iters == max_ecc + 1
    return levels, runs


def test_batch_64_roots_one_graph(ss):
    e = graphgen.rmat(14, 16, seed=21)
    c = oracle.csr_from_edgelist(e)
    G = ss.Graph.from_edgelist(e)
    roots = graphgen.pick_roots(e, 64, seed=22)[None, :]
    for mode in (0, 1, 2):
        for split in (0, 64, 1024):
            G.set_tune(split_len=split, lds_kib=32 if split == 64 else 0,
                       max_groups=128 if split == 64 else 0)
            note("batch", mode, split)
            levels, _ = _check_batch(G, [e], [c], roots, slimwork=mode, level_cap=32)
    # per-level discovered rows are counted
    assert levels["discovered"].sum() > 0


def test_batch_unused_slots_duplicates_and_few_roots(ss):
    e = graphgen.er(3000, 9000, seed=23)   # sparse: several components
    c = oracle.csr_from_edgelist(e)
    G = ss.Graph.from_edgelist(e)
    r = graphgen.pick_roots(e, 10, seed=24)
    roots = np.full((1, 64), -1, np.int32)
    roots[0, ::7] = r
    roots[0, 63] = r[0]          # the same root in two slots
    _check_batch(G, [e], [c], roots)
    _check_batch(G, [e], [c], r[None, :5].astype(np.int32))
    iso = np.array([[int(np.argmin(c.degree))]], np.int32)  # an isolated vertex
    _check_batch(G, [e], [c], iso)


def test_multi_graph_union(ss):
    graphs = [graphgen.er(int(n), int(4 * n), seed=100 + i)
              for i, n in enumerate([70, 64, 1, 300, 1000, 5000])]
    graphs.append(graphgen.EdgeList(50, np.arange(49, dtype=np.int32),
                                    np.arange(1, 50, dtype=np.int32), "path50"))
    graphs.append(graphgen.rmat(11, 8, seed=7))
    csrs = [oracle.csr_from_edgelist(g) for g in graphs]
    G = ss.Graph.from_many(graphs)
    ns, off = G.parts()
    assert list(ns) == [g.n for g in graphs]
    rpg = 64
    roots = np.full((len(graphs), rpg), -1, np.int32)
    for i, g in enumerate(graphs):
        rr = graphgen.pick_roots(g, rpg, seed=200 + i)
        roots[i, :len(rr)] = rr
        if len(rr) == 0:
            roots[i, 0] = 0
    for split in (0, 128):
        G.set_tune(split_len=split)
        note("multi", split)
        _check_batch(G, graphs, csrs, roots)
    # single-root BFS on the union sees one graph with union IDs
    import torch
    big = oracle.csr(G.n, np.concatenate([g.src + o for g, o in zip(graphs, off)]).astype(np.int32),
                     np.concatenate([g.dst + o for g, o in zip(graphs, off)]).astype(np.int32))
    ur = np.array([off[3] + 5, off[7] + 3, off[6]], np.int32)
    res = G.bfs(ur, "selmax")
    torch.cuda.synchronize()
    for i, r in enumerate(ur):
        ex = oracle.expected(big, int(r))
        np.testing.assert_array_equal(res.dist[i].cpu().numpy(), ex.dist)
        np.testing.assert_array_equal(res.parent[i].cpu().numpy(), ex.parent)


def test_batch_rmat_scale21_64_roots(ss):
    e = graphgen.rmat(21, 16, seed=1)
    c = oracle.csr_from_edgelist(e)
    G = ss.Graph.from_edgelist(e)
    roots = graphgen.pick_roots(e, 64, seed=1004)[None, :]
    note("s21 batch")
    _check_batch(G, [e], [c], roots, slots_to_check=[0, 1, 17, 40, 63])
    G.close()


def test_256_er_graphs_in_one_union(ss):
    graphs = graphgen.er_set(256, seed=3)
    csrs = [oracle.csr_from_edgelist(g) for g in graphs]
    G = ss.Graph.from_many(graphs)
    roots = np.full((256, 64), -1, np.int32)
    for i, g in enumerate(graphs):
        rr = graphgen.pick_roots(g, 64, seed=5000 + i)
        roots[i, :len(rr)] = rr
    note("256 ER graphs, n total", G.n)
    _check_batch(G, graphs, csrs, roots, slots_to_check=[0, 21, 63])
    G.close()


def test_autotune_keeps_results_and_caches(ss):
    import torch
    e = graphgen.rmat(13, 16, seed=31)
    c = oracle.csr_from_edgelist(e)
    G = ss.Graph.from_edgelist(e)
    roots = graphgen.pick_roots(e, 4, seed=32)
    r = G.autotune(roots, "selmax", repeats=1, force=True)
    assert r["evaluated"] > 10 and not r["from_cache"]
    assert r["best_ms"] <= r["before_ms"] * 1.0001
    assert G.get_tune() == r["best"]
    res = G.bfs(roots, "selmax")
    torch.cuda.synchronize()
    for i, rt in enumerate(roots):
        ex = oracle.expected(c, int(rt))
        np.testing.assert_array_equal(res.dist[i].cpu().numpy(), ex.dist)
        np.testing.assert_array_equal(res.parent[i].cpu().numpy(), ex.parent)
    G2 = ss.Graph.from_edgelist(e)
    r2 = G2.autotune(roots, "selmax")
    assert r2["from_cache"] and r2["best"] == r["best"]
    rb = G.autotune(roots[None, :], batched=True, repeats=1, force=True)
    assert rb["evaluated"] > 10
    _check_batch(G, [e], [c], roots[None, :].astype(np.int32))


def test_persistent_launch_batched_and_single_root(ss):
    import torch
    graphs = [graphgen.rmat(12, 16, seed=51), graphgen.er(3000, 20000, seed=52),
              graphgen.EdgeList(700, np.arange(699, dtype=np.int32),
                                np.arange(1, 700, dtype=np.int32), "path700")]
    csrs = [oracle.csr_from_edgelist(g) for g in graphs]
    G = ss.Graph.from_many(graphs)
    R = np.full((3, 64), -1, np.int32)
    for i, g in enumerate(graphs):
        rr = graphgen.pick_roots(g, 64, seed=53 + i)
        R[i, :len(rr)] = rr
    for split, lds in ((0, 0), (64, 32)):
        G.set_tune(split_len=split, lds_kib=lds, max_groups=0)
        note("persistent batch", split, lds)
        levels, runs = _check_batch(G, graphs, csrs, R, persistent=True, level_cap=800,
                                    timing=True)
        assert runs["launches"] == 1
    # single root, every semiring, persistent
    for i, (g, c) in enumerate(zip(graphs, csrs)):
        Gs = ss.Graph.from_edgelist(g)
        roots = graphgen.pick_roots(g, 3, seed=60 + i)
        for semi in ("tropical", "real", "boolean", "selmax"):
            note("persistent single", g.name, semi)
            res = Gs.bfs(roots, semi, persistent=True)
            torch.cuda.synchronize()
            for j, r in enumerate(roots):
                ex = oracle.expected(c, int(r))
                np.testing.assert_array_equal(res.dist[j].cpu().numpy(), ex.dist)
                assert int(res.iterations[j]) == ex.iterations
                if semi == "selmax":
                    np.testing.assert_array_equal(res.parent[j].cpu().numpy(), ex.parent)
                if semi == "real":
                    np.testing.assert_array_equal(res.real_val[j].cpu().numpy(), ex.real_val)
        if g.name == "path700":  # the level cap is reported, not hung on
            with pytest.raises(ss.SlimSellError) as ei:
                Gs.bfs([0], "boolean", persistent=True, max_levels=2)
            assert ei.value.code == -5
        Gs.close()
    G.close()
