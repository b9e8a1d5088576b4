"""GPU tests of the DP transformation (parents from distances, Section II-C):
bit-exact against the oracle's max-ID parents for every semiring, every
split length (pieces combine by atomicMax) and distances from the batched
SpMM."""
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


def _graphs():
    return [graphgen.rmat(13, 16, seed=71),
            graphgen.er(5000, 9000, seed=72),            # many components and isolated vertices
            graphgen.grid(50, 40, 0.05, seed=5),
            graphgen.EdgeList(257, np.zeros(256, np.int32), np.arange(1, 257, dtype=np.int32),
                              "star257")]


@pytest.mark.parametrize("split", [0, 64, 256])
def test_dp_parents_every_semiring(ss, split):
    import torch
    for e in _graphs():
        g = oracle.csr_from_edgelist(e)
        G = ss.Graph.from_edgelist(e)
        G.set_tune(split_len=split)
        roots = graphgen.pick_roots(e, 3, seed=73)
        exs = [oracle.expected(g, int(r)) for r in roots]
        for semi in ("tropical", "real", "boolean", "selmax"):
            note(e.name, "split", split, semi)
            res = G.bfs(roots, semi, dp=True)
            torch.cuda.synchronize()
            for i, ex in enumerate(exs):
                np.testing.assert_array_equal(res.dist[i].cpu().numpy(), ex.dist)
                np.testing.assert_array_equal(res.parent[i].cpu().numpy(), ex.parent)
            if semi == "selmax":
                # the DP pass on sel-max's distances reproduces its own parents
                p2 = G.dp_parents(res.dist)
                torch.cuda.synchronize()
                assert torch.equal(p2, res.parent)
        G.close()


def test_dp_on_batched_distances_and_edge_cases(ss):
    import torch
    e = graphgen.rmat(12, 16, seed=74)
    g = oracle.csr_from_edgelist(e)
    G = ss.Graph.from_edgelist(e)
    roots = graphgen.pick_roots(e, 64, seed=75)
    dist, _, _, _ = G.bfs_batch(roots)
    par = G.dp_parents(dist)
    torch.cuda.synchronize()
    P = par.view(64, -1).cpu().numpy()
    for i in range(0, 64, 7):
        ex = oracle.expected(g, int(roots[i]))
        np.testing.assert_array_equal(P[i], ex.parent)
    # an isolated root: only itself
    deg = G.degrees()
    iso = np.flatnonzero(deg == 0)
    if iso.size:
        res = G.bfs([int(iso[0])], "boolean", dp=True)
        p = res.parent[0].cpu().numpy()
        assert p[iso[0]] == iso[0] and np.count_nonzero(p >= 0) == 1
    # arbitrary (non-BFS) input stays in bounds and yields valid IDs or -1
    junk = torch.randint(-3, 40, (G.n,), dtype=torch.int32, device="cuda")
    pj = G.dp_parents(junk)
    torch.cuda.synchronize()
    pj = pj.cpu().numpy()
    assert pj.min() >= -1 and pj.max() < G.n
    with pytest.raises(ValueError):
        G.dp_parents(torch.zeros(G.n + 1, dtype=torch.int32, device="cuda"))
    G.close()


@pytest.mark.parametrize("no_alloc", [False, True], ids=["bfs", "noalloc"])
def test_dp_pass_writes_every_distance_and_parent(ss, no_alloc):
    """Without real values, the transformation's last pass writes the
    distances as well as the parents: outputs filled with garbage first must
    come back whole and equal to the oracle's, for every semiring that needs
    the transformation, on a graph with isolated and unreachable vertices."""
    import torch
    e = graphgen.er(5000, 9000, seed=76)
    g = oracle.csr_from_edgelist(e)
    G = ss.Graph.from_edgelist(e)
    roots = graphgen.pick_roots(e, 3, seed=77)
    exs = [oracle.expected(g, int(r)) for r in roots]
    try:
        for semi in ("tropical", "real", "boolean"):
            note("garbage-filled outputs", semi, "noalloc" if no_alloc else "bfs")
            dist = torch.full((len(roots), G.n), -7, dtype=torch.int32, device="cuda")
            parent = torch.full_like(dist, -7)
            res = G.bfs(roots, semi, dp=True, want_real=False, dist=dist, parent=parent,
                        no_alloc=no_alloc)
            torch.cuda.synchronize()
            assert res.real_val is None
            for i, ex in enumerate(exs):
                np.testing.assert_array_equal(dist[i].cpu().numpy(), ex.dist)
                np.testing.assert_array_equal(parent[i].cpu().numpy(), ex.parent)
    finally:
        G.close()
