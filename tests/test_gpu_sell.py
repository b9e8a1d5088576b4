"""GPU tests of the Sell-C-sigma comparator (a val array streamed beside col,
Section II-D): results bit-identical to the oracle and to SlimSell."""
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


@pytest.mark.parametrize("sigma", [1, 64, 0])
def test_sell_comparator_is_exact(ss, sigma):
    import torch
    for e in (graphgen.rmat(13, 16, seed=81), graphgen.er(4000, 30000, seed=82),
              graphgen.grid(40, 30, 0.05, seed=5)):
        g = oracle.csr_from_edgelist(e)
        G = ss.Graph.from_edgelist(e, sigma=sigma)
        roots = graphgen.pick_roots(e, 2, seed=83)
        exs = [oracle.expected(g, int(r)) for r in roots]
        for split in (0, 64):
            for semi in ("tropical", "real", "boolean", "selmax"):
                note(e.name, sigma, split, semi)
                res = G.bfs(roots, semi, sell=True, split_len=split)
                torch.cuda.synchronize()
                for i, ex in enumerate(exs):
                    np.testing.assert_array_equal(res.dist[i].cpu().numpy(), ex.dist)
                    assert int(res.iterations[i]) == ex.iterations
                    if semi == "selmax":
                        np.testing.assert_array_equal(res.parent[i].cpu().numpy(), ex.parent)
                    if semi == "real":
                        np.testing.assert_array_equal(res.real_val[i].cpu().numpy(),
                                                      ex.real_val)
        for bad in (dict(schedule="heuristic"), dict(persistent=True)):
            with pytest.raises(ss.SlimSellError):
                G.bfs(roots[:1], "selmax", sell=True, **bad)
        G.close()
