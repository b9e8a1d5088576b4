"""The allocation-free entry point (slimsell_bfs_noalloc), called through the
C ABI, against slimsell_bfs: identical distances, parents, real values and
iteration counts, on two calls in a row with the second on a smaller graph
(the shared device scratch keeps the first call's contents), for every
semiring, with and without parents by the DP transformation."""
import ctypes
import sys

import numpy as np
import pytest

import graphgen

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


def _raw_noalloc(ss, G, roots, semi, dist, parent, real_val):
    """slimsell_bfs_noalloc through ctypes with caller-owned outputs."""
    import torch
    from paper_2010_09913_amd import _native
    roots = np.ascontiguousarray(roots, np.int32)
    iters = np.zeros(len(roots), np.int32)
    o = _native.BfsOpts()
    o.size = ctypes.sizeof(_native.BfsOpts)
    o.slimwork = 2
    o.split_len = -1
    o.stream = ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))
    o.iterations_out = iters.ctypes.data_as(_native.c_i32p)

    def ptr(t):
        return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p()

    rc = _native.load().slimsell_bfs_noalloc(G._h, roots.ctypes.data_as(_native.c_i32p),
                                             len(roots), ss.SEMIRINGS[semi], ctypes.byref(o),
                                             ptr(dist), ptr(parent), ptr(real_val))
    _native.check(rc)
    return iters


def _compare(ss, G, roots, semi, with_parent):
    import torch
    nr, n = len(roots), G.n
    ref = G.bfs(roots, semi, dp=with_parent and semi != "selmax",
                want_parent=with_parent)
    # outputs filled with garbage first: every element must be written
    dist = torch.full((nr, n), -7, dtype=torch.int32, device="cuda")
    parent = torch.full((nr, n), -7, dtype=torch.int32, device="cuda") if with_parent else None
    real_val = (torch.full((nr, n), -7.0, dtype=torch.float32, device="cuda")
                if semi == "real" else None)
    iters = _raw_noalloc(ss, G, roots, semi, dist, parent, real_val)
    torch.cuda.synchronize()
    assert torch.equal(dist, ref.dist), (semi, "dist")
    np.testing.assert_array_equal(iters, ref.iterations)
    if with_parent:
        assert torch.equal(parent, ref.parent), (semi, "parent")
    if semi == "real":
        assert torch.equal(real_val, ref.real_val), (semi, "real_val")


@pytest.mark.parametrize("with_parent", [False, True], ids=["dist", "parent"])
@pytest.mark.parametrize("semi", SEMIS)
def test_noalloc_matches_bfs_on_two_calls_in_a_row(ss, semi, with_parent):
    big = graphgen.rmat(16, 16, seed=11)            # 65,536 vertices, several tiles
    small = graphgen.er(3001, 12000, seed=12)       # fewer vertices than the first
    Gb = ss.Graph.from_edgelist(big, sigma=0)
    Gs = ss.Graph.from_edgelist(small, sigma=0)
    try:
        for G, e, tag in ((Gb, big, "larger"), (Gs, small, "smaller")):
            roots = graphgen.pick_roots(e, 3, seed=13)
            note(semi, "parent" if with_parent else "dist", tag, "graph, roots", roots.tolist())
            _compare(ss, G, roots, semi, with_parent)
    finally:
        Gb.close()
        Gs.close()


def test_noalloc_with_the_binding_and_a_tuned_configuration(ss):
    import torch
    e = graphgen.rmat(14, 16, seed=21)
    G = ss.Graph.from_edgelist(e, sigma=0)
    try:
        roots = graphgen.pick_roots(e, 2, seed=22)
        G.set_tune(split_len=1024, waves_per_group=8)
        a = G.bfs(roots, "selmax")
        b = G.bfs(roots, "selmax", no_alloc=True)
        torch.cuda.synchronize()
        assert torch.equal(a.dist, b.dist) and torch.equal(a.parent, b.parent)
        np.testing.assert_array_equal(a.iterations, b.iterations)
        # a split length whose work units were never prepared is refused
        with pytest.raises(ss.SlimSellError, match="no work units"):
            G.bfs(roots, "selmax", split_len=96, no_alloc=True)
    finally:
        G.close()


def test_noalloc_refuses_what_needs_allocation_or_too_much_scratch(ss):
    e = graphgen.er(4000, 8000, seed=31)
    G = ss.Graph.from_edgelist(e, sigma=0)
    try:
        for kw in (dict(timing=True), dict(level_cap=4), dict(schedule="heuristic"),
                   dict(persistent=True), dict(sell=True)):
            with pytest.raises(ss.SlimSellError, match="allocation-free"):
                G.bfs([0], "boolean", no_alloc=True, **kw)
    finally:
        G.close()
    # 3.5 million rows of the real semiring need 21 B each: beyond 64 MiB
    n = 3_500_000
    src = np.arange(0, 2000, dtype=np.int32)
    dst = src + 1
    Gl = ss.Graph(src, dst, n, sigma=0)
    try:
        with pytest.raises(ss.SlimSellError, match="bytes of scratch"):
            Gl.bfs([0], "real", no_alloc=True)
        # sel-max needs about 13 B per row: fits
        r = Gl.bfs([0], "selmax", no_alloc=True)
        d = r.dist[0].cpu().numpy()
        assert d[0] == 0 and d[2000] == 2000 and d[2001] == -1
    finally:
        Gl.close()
