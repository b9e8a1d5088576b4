"""GPU tests of the frontier-summary filter of plain single-root runs.

Each level records one bit per 64-row chunk that gained frontier rows; the
next level reads a term from memory only when its row's chunk has one.  The
filter must not change any result: every semiring, SlimWork mode and split
length gives the oracle's distances, parents and real values with the filter
on and off, on graphs whose frontiers are small for many levels (a grid, a
path) as well as on skewed ones, in the launch-per-level and the persistent
form, and with and without the LDS-staged prefix.
"""
import sys

import numpy as np
import pytest

import graphgen
import oracle

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


def _graphs():
    n = 3000
    path = graphgen.EdgeList(n, np.arange(n - 1, dtype=np.int32), np.arange(1, n, dtype=np.int32),
                             "path3000")
    return [graphgen.rmat(13, 16, seed=81), graphgen.grid(60, 50, 0.05, seed=82), path,
            graphgen.er(6000, 12000, seed=83)]


def _compare(res, exs, semi):
    for i, ex in enumerate(exs):
        assert int(res.iterations[i]) == ex.iterations
        np.testing.assert_array_equal(res.dist[i].cpu().numpy(), ex.dist)
        if semi == "selmax":
            np.testing.assert_array_equal(res.parent[i].cpu().numpy(), ex.parent)
        if semi == "real":
            np.testing.assert_array_equal(res.real_val[i].cpu().numpy(), ex.real_val)


@pytest.mark.parametrize("lds_kib", [64, 0])
def test_filter_on_and_off_match_the_oracle(ss, lds_kib):
    import torch
    for e in _graphs():
        g = oracle.csr_from_edgelist(e)
        G = ss.Graph.from_edgelist(e)
        roots = graphgen.pick_roots(e, 3, seed=84)
        exs = [oracle.expected(g, int(r)) for r in roots]
        for semi in SEMIS:
            for slimwork in (0, 1, 2):
                for split in (0, 64):
                    G.set_tune(split_len=split, lds_kib=lds_kib)
                    outs = []
                    for summary in (True, False):
                        note(e.name, semi, "slimwork", slimwork, "split", split, "lds", lds_kib,
                             "summary", summary)
                        res = G.bfs(roots, semi, slimwork=slimwork, summary=summary)
                        torch.cuda.synchronize()
                        _compare(res, exs, semi)
                        outs.append(res.iterations.copy())
                    np.testing.assert_array_equal(outs[0], outs[1])
        G.close()


def test_filter_in_the_persistent_form_and_repeated_runs(ss):
    import torch
    e = graphgen.grid(70, 40, 0.05, seed=85)
    g = oracle.csr_from_edgelist(e)
    G = ss.Graph.from_edgelist(e)
    roots = graphgen.pick_roots(e, 4, seed=86)
    exs = [oracle.expected(g, int(r)) for r in roots]
    for semi in SEMIS:
        note("persistent", semi)
        res = G.bfs(roots, semi, persistent=True)
        torch.cuda.synchronize()
        _compare(res, exs, semi)
        # the summaries of one run must not leak into the next
        res = G.bfs(roots[::-1], semi)
        torch.cuda.synchronize()
        _compare(res, exs[::-1], semi)
    G.close()


def test_batched_masks_with_and_without_the_summary(ss):
    # the batched SpMM keeps a summary of chunks whose rows gained root bits;
    # distances with it on and off must both be the oracle's, on one graph
    # and on a union of uneven graphs (persistent form included)
    import torch
    graphs = [graphgen.er(int(n), int(4 * n), seed=90 + i) for i, n in enumerate([70, 1, 3000])]
    graphs.append(graphgen.grid(40, 30, 0.05, seed=93))
    graphs.append(graphgen.rmat(12, 16, seed=94))
    csrs = [oracle.csr_from_edgelist(g) for g in graphs]
    G = ss.Graph.from_many(graphs)
    ns, off = G.parts()
    rpg = 64
    roots = np.full((len(graphs), rpg), -1, np.int32)
    for i, g in enumerate(graphs):
        rr = graphgen.pick_roots(g, rpg, seed=300 + i)
        roots[i, :len(rr)] = rr
        if len(rr) == 0:
            roots[i, 0] = 0
    for summary in (True, False):
        for persistent in (False, True):
            note("batched summary", summary, "persistent", persistent)
            dist, _, _, _ = G.bfs_batch(roots, summary=summary, persistent=persistent)
            torch.cuda.synchronize()
            d = dist.cpu().numpy()
            for i, c in enumerate(csrs):
                blk = d[rpg * off[i]: rpg * (off[i] + ns[i])].reshape(rpg, ns[i])
                for b in (0, 1, 31, 63):
                    r = int(roots[i, b])
                    if r < 0:
                        assert np.all(blk[b] == -1)
                    else:
                        np.testing.assert_array_equal(blk[b], oracle.bfs(c, r))
    G.close()
