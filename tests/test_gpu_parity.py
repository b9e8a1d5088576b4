"""GPU parity: every HIP BFS form against the CPU oracle, element by element.

Distances and parents must be bit-exact; real-semiring fp32 values must match
with tolerance 0 (they are small integers, exact in fp32).  Iteration counts
must equal eccentricity + 1 and per-level discovered counts must equal the
oracle's literal semiring stepping.  Inputs are seeded synthetic graphs of the
shapes the paper evaluates (Kronecker/R-MAT, Erdos-Renyi, grids) plus
closed-form families and all 5-vertex graphs.
"""
import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

SEMIS = ["tropical", "real", "boolean", "selmax"]
OR_SEMI = {"tropical": oracle.TROPICAL, "real": oracle.REAL, "boolean": oracle.BOOLEAN,
           "selmax": oracle.SELMAX}


@pytest.fixture(scope="module")
def ss():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2010_09913_amd as mod
    return mod


def note(*a):
    print(*a, file=sys.stderr, flush=True)


_CACHE = {}


def _graph(ss, e, sigma=0):
    key = (e.name, e.n, e.m, sigma)
    if key not in _CACHE:
        _CACHE[key] = ss.Graph.from_edgelist(e, sigma=sigma)
    return _CACHE[key]


def _csr(e):
    key = ("csr", e.name, e.n, e.m)
    if key not in _CACHE:
        _CACHE[key] = oracle.csr_from_edgelist(e)
    return _CACHE[key]


def _check(ss, G, g, roots, semi, **kw):
    import torch
    res = G.bfs(roots, semi, **kw)
    torch.cuda.synchronize()
    dist = res.dist.cpu().numpy()
    par = res.parent.cpu().numpy() if res.parent is not None else None
    rv = res.real_val.cpu().numpy() if res.real_val is not None else None
    for i, r in enumerate(np.atleast_1d(roots)):
        ex = oracle.expected(g, int(r))
        np.testing.assert_array_equal(dist[i], ex.dist, err_msg=f"{semi} root {r} dist {kw}")
        assert res.iterations[i] == ex.iterations, (semi, r, kw)
        if res.levels is not None:
            cap = res.levels["discovered"].shape[1]
            hist = np.bincount(ex.dist[ex.dist > 0], minlength=ex.iterations + 1)[1:]
            hist = np.concatenate([hist, np.zeros(max(0, cap - len(hist)), np.int64)])[:cap]
            np.testing.assert_array_equal(res.levels["discovered"][i], hist)
            cells = res.levels["active_cells"][i]
            assert np.all(cells[:ex.iterations] >= 0) and np.all(cells[ex.iterations:] == 0)
        if semi == "selmax":
            np.testing.assert_array_equal(par[i], ex.parent, err_msg=f"root {r} parent {kw}")
        if semi == "real":
            np.testing.assert_array_equal(rv[i], ex.real_val, err_msg=f"root {r} real {kw}")
    return res


# ------------------------------------------------------------ configuration 1

def test_rmat_scale12_tropical_from_the_max_degree_root(ss):
    e = graphgen.rmat(12, 16, seed=1)
    g = _csr(e)
    root = int(np.argmax(g.degree))  # argmax takes the smallest ID among ties
    G = _graph(ss, e, sigma=4096)
    note("c1 root", root)
    res = _check(ss, G, g, [root], "tropical", level_cap=64, timing=True)
    ref = oracle.semiring_bfs(g, root, oracle.TROPICAL)
    np.testing.assert_array_equal(res.frontier[:ref.iterations], ref.frontier_sizes)
    # without SlimWork every level streams every non-empty chunk
    L = ss.layout_build(e.src, e.dst, e.n, sigma=4096)
    res = G.bfs([root], "tropical", slimwork=0, split_len=0, level_cap=64, timing=True)
    it = int(res.iterations[0])
    assert np.all(res.levels["active_cells"][0][:it] == L.cells)
    assert np.all(res.levels["active_chunks"][0][:it] == (L.cl > 0).sum())
    assert np.all(res.levels["max_active_cl"][0][:it] == L.max_cl)
    assert np.all(res.levels["ms"][0][:it] > 0)
    assert res.runs["launches"][0] >= it + 1
    assert res.runs["bfs_ms"][0] >= res.runs["kernel_ms"][0] > 0


# ---------------------------------------------------- small-matrix sweeps

@pytest.mark.parametrize("sigma", [1, 64, 1024, 0])
@pytest.mark.parametrize("kind", ["rmat", "er"])
def test_all_semirings_slimwork_and_splits(ss, kind, sigma):
    e = graphgen.rmat(12, 16, seed=7) if kind == "rmat" else graphgen.er(3000, 24000, seed=8)
    g = _csr(e)
    G = _graph(ss, e, sigma=sigma)
    roots = graphgen.pick_roots(e, 3, seed=9)
    for semi in SEMIS:
        ref = oracle.semiring_bfs(g, int(roots[-1]), OR_SEMI[semi])
        for slimwork in (0, 1, 2):
            for split in (0, 16, 64, 256):
                note(kind, sigma, semi, slimwork, split)
                res = _check(ss, G, g, roots, semi, slimwork=slimwork, split_len=split,
                             level_cap=64)
                np.testing.assert_array_equal(res.levels["discovered"][-1][:ref.iterations],
                                              ref.frontier_sizes)


@pytest.mark.parametrize("waves", [1, 2, 4, 8, 16])
def test_workgroup_shapes_give_identical_results(ss, waves):
    e = graphgen.rmat(13, 16, seed=3)
    g = _csr(e)
    G = _graph(ss, e)
    roots = graphgen.pick_roots(e, 4, seed=5)
    for semi in SEMIS:
        note("waves", waves, semi)
        _check(ss, G, g, roots, semi, waves_per_group=waves, split_len=128)


# ------------------------------------------------------------ closed forms

def _pairs_graph(n, pairs, name):
    pairs = np.asarray(pairs, np.int32).reshape(-1, 2)
    return graphgen.EdgeList(n, pairs[:, 0].copy(), pairs[:, 1].copy(), name)


FAMILIES = {
    "path": lambda: _pairs_graph(700, [(i, i + 1) for i in range(699)], "path700"),
    "cycle": lambda: _pairs_graph(257, [(i, (i + 1) % 257) for i in range(257)], "cycle257"),
    "star": lambda: _pairs_graph(5000, [(0, i) for i in range(1, 5000)], "star5000"),
    "complete": lambda: _pairs_graph(
        150, [(i, j) for i in range(150) for j in range(i + 1, 150)], "k150"),
    "hypercube": lambda: _pairs_graph(
        1024, [(v, v ^ (1 << b)) for v in range(1024) for b in range(10) if v < v ^ (1 << b)],
        "q10"),
    "grid": lambda: graphgen.grid(64, 48, 0.0),
    "grid_cut": lambda: graphgen.grid(80, 70, 0.05, seed=5),
}


@pytest.mark.parametrize("family", list(FAMILIES))
def test_closed_form_families(ss, family):
    e = FAMILIES[family]()
    g = _csr(e)
    G = _graph(ss, e)
    roots = np.unique(np.array([0, e.n - 1, e.n // 2, e.n // 3], np.int32))
    for semi in SEMIS:
        for split in (0, 32):
            note(family, semi, split)
            _check(ss, G, g, roots, semi, split_len=split)


def test_all_five_vertex_graphs_as_one_union(ss):
    import itertools
    pairs = list(itertools.combinations(range(5), 2))
    src, dst = [], []
    for mask in range(1 << len(pairs)):
        base = 5 * mask
        for i, (a, b) in enumerate(pairs):
            if mask >> i & 1:
                src.append(base + a)
                dst.append(base + b)
    e = graphgen.EdgeList(5 * 1024, np.array(src, np.int32), np.array(dst, np.int32), "all5")
    g = _csr(e)
    for sigma in (0, 1):
        G = _graph(ss, e, sigma=sigma)
        roots = np.arange(0, e.n, 1, dtype=np.int32)
        for semi in SEMIS:
            note("all5", sigma, semi)
            _check(ss, G, g, roots[:: (1 if semi == "selmax" else 7)], semi, split_len=0)


# ------------------------------------------------------------ edge cases

def test_edge_cases(ss):
    import torch
    from paper_2010_09913_amd import _native
    # a single vertex, no edges
    G = ss.Graph(np.zeros(0, np.int32), np.zeros(0, np.int32), 1)
    r = G.bfs([0], "selmax")
    assert r.dist.cpu().tolist() == [[0]] and r.parent.cpu().tolist() == [[0]]
    assert r.iterations.tolist() == [1]
    # empty graph with a ragged vertex count, isolated roots
    G = ss.Graph(np.zeros(0, np.int32), np.zeros(0, np.int32), 100)
    for semi in SEMIS:
        r = G.bfs([7, 99], semi)
        d = r.dist.cpu().numpy()
        assert d[0, 7] == 0 and d[1, 99] == 0 and (d == -1).sum() == 2 * 99
    # self-loops and duplicates only
    e = _pairs_graph(130, [(3, 3), (3, 4), (4, 3), (3, 4), (129, 129)], "dups")
    _check(ss, _graph(ss, e), _csr(e), [3, 129, 4], "selmax")
    # argument errors
    G = ss.Graph([0, 1], [1, 2], 3)
    for kw, code in [(dict(roots=[3]), _native.SS_EINVAL), (dict(roots=[-1]), _native.SS_EINVAL),
                     (dict(roots=[0], waves_per_group=3), _native.SS_EINVAL),
                     (dict(roots=[0], split_len=-2), _native.SS_EINVAL)]:
        with pytest.raises(ss.SlimSellError) as ei:
            G.bfs(kw.pop("roots"), "tropical", **kw)
        assert ei.value.code == code
    # parents with a non-sel-max semiring come from the DP transformation
    par = torch.full((1, 3), -7, dtype=torch.int32, device="cuda")
    G.bfs([0], "tropical", parent=par)
    assert par.cpu().tolist() == [[0, 0, 1]]
    with pytest.raises(ss.SlimSellError):
        G.bfs([0], "boolean", real_val=torch.empty((1, 3), dtype=torch.float32, device="cuda"))
    # the level cap is reported, not hung on
    e = _pairs_graph(50, [(i, i + 1) for i in range(49)], "path50")
    Gp = _graph(ss, e)
    with pytest.raises(ss.SlimSellError) as ei:
        Gp.bfs([0], "boolean", max_levels=10)
    assert ei.value.code == _native.SS_EITER
    r = Gp.bfs([0], "boolean", max_levels=50)
    assert r.iterations.tolist() == [50]
    # the graph is still usable after an error
    _check(ss, Gp, _csr(e), [0, 25], "tropical")


# ------------------------------------------------- configurations 2 and 3

def test_rmat_scale20_all_semirings(ss):
    e = graphgen.rmat(20, 16, seed=1)
    g = _csr(e)
    G = _graph(ss, e, sigma=1 << 14)
    roots = graphgen.pick_roots(e, 16, seed=1001)
    for semi in SEMIS:
        note("s20", semi)
        _check(ss, G, g, roots, semi, slimwork=2)
    for mode in (0, 1):
        note("s20 selmax slimwork", mode)
        _check(ss, G, g, roots[:4], "selmax", slimwork=mode)
    ref = oracle.semiring_bfs(g, int(roots[0]), oracle.BOOLEAN)
    res = G.bfs(roots[:1], "boolean", level_cap=64)
    np.testing.assert_array_equal(res.frontier[:ref.iterations], ref.frontier_sizes)
    # m_cc from the library's degrees equals the oracle's
    deg = G.degrees()
    np.testing.assert_array_equal(deg, g.degree)


@pytest.mark.parametrize("kind", ["rmat", "er"])
def test_scale22_selmax_split_sweep(ss, kind):
    if kind == "rmat":
        e = graphgen.rmat(22, 16, seed=1)
        seed = 1002
    else:
        e = graphgen.er(1 << 22, 16 << 22, seed=2)
        seed = 1003
    g = _csr(e)
    G = _graph(ss, e, sigma=0)
    roots = graphgen.pick_roots(e, 64, seed=seed)[:3]
    for split in (256, 1024, 4096):
        note("s22", kind, split)
        _check(ss, G, g, roots, "selmax", slimwork=2, split_len=split)
    _check(ss, G, g, roots[:1], "selmax", slimwork=1, split_len=1024)
    _CACHE.clear()


@pytest.mark.parametrize("tune", [
    dict(unroll=4), dict(unroll=16), dict(max_groups=64), dict(max_groups=7, waves_per_group=2),
    dict(pack_cols=0), dict(pack_cols=40, split_len=96), dict(split_len=0, pack_cols=0),
    dict(lds_kib=64, max_groups=64), dict(lds_kib=16, max_groups=512, waves_per_group=16),
    dict(lds_kib=32, unroll=4),
])
def test_launch_configurations_give_identical_results(ss, tune):
    e = graphgen.rmat(13, 16, seed=11)
    g = _csr(e)
    G = ss.Graph.from_edgelist(e, sigma=0)
    G.set_tune(**tune)
    roots = graphgen.pick_roots(e, 3, seed=12)
    for semi in SEMIS:
        for mode in (1, 2):
            note("tune", tune, semi, mode)
            _check(ss, G, g, roots, semi, slimwork=mode)
    with pytest.raises(ss.SlimSellError):
        G.set_tune(unroll=3)
    G.close()


def test_repeated_runs_reuse_the_prepared_work_lists(ss):
    """Repeated BFS calls on one graph reuse the per-wavefront unit lists
    (built once per graph, split length and grid): device memory stays flat
    over many calls, and the results stay exact."""
    import torch
    e = graphgen.rmat(20, 16, seed=9)
    g = oracle.csr_from_edgelist(e)
    G = ss.Graph.from_edgelist(e, sigma=0)
    root = int(graphgen.pick_roots(e, 1, seed=91)[0])
    ex = oracle.expected(g, root)
    try:
        for _ in range(3):  # warm-up: work lists, workspace, torch's cache
            G.bfs([root], "selmax")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for _ in range(60):
            res = G.bfs([root], "selmax")
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        note("free device memory", free0, "->", free1)
        assert free0 - free1 < (4 << 20), (free0, free1)
        np.testing.assert_array_equal(res.dist[0].cpu().numpy(), ex.dist)
        np.testing.assert_array_equal(res.parent[0].cpu().numpy(), ex.parent)
    finally:
        G.close()
