"""Pins of the CPU oracle against facts it does not compute itself.

Every check here comes from outside the oracle's own code path: Floyd-Warshall
and dense textbook semiring products on tiny graphs (the O(D n^2) BFS-SpMV row
of Table "compar"), closed forms of distances, parents and real-semiring values
on structured graphs, BFS invariants, and the negation example printed in
Section II-A.  A dropped term, a wrong sign, index or tie-break in the oracle
fails at least one of them.
"""
import itertools

import numpy as np
import pytest

import graphgen
import oracle

SEMIRINGS = [oracle.TROPICAL, oracle.REAL, oracle.BOOLEAN, oracle.SELMAX]


def _csr_from_pairs(n, pairs):
    pairs = np.asarray(pairs, np.int32).reshape(-1, 2)
    return oracle.csr(n, pairs[:, 0].copy(), pairs[:, 1].copy())


def _all_checks(g, root, exp_dist, exp_parent=None, exp_real=None):
    d = oracle.bfs(g, root)
    np.testing.assert_array_equal(d, exp_dist)
    ex = oracle.expected(g, root)
    if exp_parent is not None:
        np.testing.assert_array_equal(ex.parent, exp_parent)
    if exp_real is not None:
        np.testing.assert_array_equal(ex.real_val, np.asarray(exp_real, np.float32))
    for s in SEMIRINGS:
        r = oracle.semiring_bfs(g, root, s)
        np.testing.assert_array_equal(r.dist, exp_dist, err_msg=f"semiring {s}")
        assert r.iterations == int(exp_dist.max()) + 1
        if s == oracle.SELMAX and exp_parent is not None:
            np.testing.assert_array_equal(r.parent, exp_parent)
        if s == oracle.REAL and exp_real is not None:
            np.testing.assert_array_equal(r.real_val, np.asarray(exp_real, np.float32))


# ---------------------------------------------------------------- Section II-A

def test_negation_example_from_paper():
    # Section II-A prints NOT((0, 7, 0)^T) = (1, 0, 1)^T.
    np.testing.assert_array_equal(oracle.lneg([0.0, 7.0, 0.0]), [1.0, 0.0, 1.0])
    np.testing.assert_array_equal(oracle.lneg(oracle.lneg([0.0, 7.0, -2.5, 0.0])),
                                  [0.0, 1.0, 1.0, 0.0])


# ------------------------------------------------------------ canonicalisation

def test_csr_is_the_simple_undirected_graph():
    g = graphgen.rmat(10, 8, seed=3)
    c = oracle.csr_from_edgelist(g)
    u = np.concatenate([g.src, g.dst]).astype(np.int64)
    v = np.concatenate([g.dst, g.src]).astype(np.int64)
    keep = u != v
    keys = np.unique(u[keep] * g.n + v[keep])
    rows = np.repeat(np.arange(g.n), np.diff(c.rowptr))
    np.testing.assert_array_equal(rows.astype(np.int64) * g.n + c.adj, keys)


# ------------------------------------------------------------- brute force

def _floyd_warshall(n, adjm):
    inf = 10 ** 9
    d = np.full((n, n), inf, np.int64)
    d[adjm] = 1
    np.fill_diagonal(d, 0)
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    d[d >= inf] = -1
    return d


def _dense_semiring(n, adjm, root, s):
    """Textbook dense products (explicit matrices, O(n^2) per step)."""
    A = adjm.astype(np.float64)
    INF = np.inf
    d = np.full(n, -1, np.int64)
    d[root] = 0
    par = np.full(n, -1, np.int64)
    par[root] = root
    real = np.zeros(n)
    real[root] = 1.0
    if s == oracle.TROPICAL:
        Ap = np.where(adjm, 1.0, INF)
        np.fill_diagonal(Ap, 0.0)
        f = np.full(n, INF)
        f[root] = 0
        for _ in range(n + 1):
            fn = np.min(Ap + f[None, :], axis=1)
            if np.array_equal(fn, f):
                break
            f = fn
        d = np.where(np.isinf(f), -1, f).astype(np.int64)
        return d, None, None
    if s in (oracle.REAL, oracle.BOOLEAN):
        f = np.zeros(n)
        f[root] = 1
        seen = f.copy()
        for k in range(1, n + 2):
            x = A @ f
            new = (x != 0) & (seen == 0)
            if not new.any():
                break
            d[new] = k
            real[new] = x[new]
            f = new.astype(np.float64)
            seen += f
        return d, None, real
    # sel-max: values are 1-based IDs, product is max_j A_ij * x_j
    x = np.zeros(n)
    x[root] = root + 1
    p = x.copy()
    seen = np.zeros(n)
    seen[root] = 1
    for k in range(1, n + 2):
        xk = np.max(A * x[None, :], axis=1)
        new = (xk != 0) & (seen == 0)
        p = np.where(p != 0, p, xk)
        if not new.any():
            break
        d[new] = k
        seen[new] = 1
        x = np.where(xk != 0, np.arange(1, n + 1), 0).astype(np.float64)
    par = np.where(p != 0, p - 1, -1).astype(np.int64)
    return d, par, None


def test_exhaustive_five_vertex_graphs_against_floyd_warshall_and_dense_products():
    n = 5
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        adjm = np.zeros((n, n), bool)
        for a, b in edges:
            adjm[a, b] = adjm[b, a] = True
        g = _csr_from_pairs(n, edges if edges else np.zeros((0, 2), np.int32))
        fw = _floyd_warshall(n, adjm)
        for root in range(n):
            d = oracle.bfs(g, root)
            np.testing.assert_array_equal(d, fw[root])
            ex = oracle.expected(g, root)
            dd, pp, _ = _dense_semiring(n, adjm, root, oracle.SELMAX)
            np.testing.assert_array_equal(ex.parent, pp)
            _, _, rr = _dense_semiring(n, adjm, root, oracle.REAL)
            np.testing.assert_array_equal(ex.real_val, rr.astype(np.float32))
            for s in SEMIRINGS:
                r = oracle.semiring_bfs(g, root, s)
                np.testing.assert_array_equal(r.dist, fw[root])
                assert r.iterations == int(fw[root].max()) + 1
                if s == oracle.SELMAX:
                    np.testing.assert_array_equal(r.parent, pp)
                if s == oracle.REAL:
                    np.testing.assert_array_equal(r.real_val, rr.astype(np.float32))


@pytest.mark.parametrize("seed", range(12))
def test_dense_products_on_random_eight_vertex_graphs(seed):
    rng = np.random.default_rng(seed)
    n = 8
    adjm = np.triu(rng.random((n, n)) < 0.3, 1)
    adjm = adjm | adjm.T
    edges = np.argwhere(np.triu(adjm, 1))
    g = _csr_from_pairs(n, edges if len(edges) else np.zeros((0, 2), np.int32))
    for root in range(n):
        for s in SEMIRINGS:
            dd, pp, rr = _dense_semiring(n, adjm, root, s)
            r = oracle.semiring_bfs(g, root, s)
            np.testing.assert_array_equal(r.dist, dd)
            if pp is not None:
                np.testing.assert_array_equal(r.parent, pp)
            if s == oracle.REAL:
                np.testing.assert_array_equal(r.real_val, rr.astype(np.float32))


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n,root", [(1, 0), (2, 1), (7, 0), (7, 3), (64, 63), (130, 17)])
def test_path(n, root):
    g = _csr_from_pairs(n, [(i, i + 1) for i in range(n - 1)] or np.zeros((0, 2)))
    i = np.arange(n)
    dist = np.abs(i - root)
    par = np.where(i > root, i - 1, np.where(i < root, i + 1, root))
    real = np.ones(n)
    _all_checks(g, root, dist, par, real)
    if root == 0:
        assert oracle.semiring_bfs(g, root, oracle.TROPICAL).iterations == n


@pytest.mark.parametrize("n,root", [(3, 0), (8, 2), (9, 4), (100, 99)])
def test_cycle(n, root):
    g = _csr_from_pairs(n, [(i, (i + 1) % n) for i in range(n)])
    i = np.arange(n)
    a = np.abs(i - root)
    dist = np.minimum(a, n - a)
    real = np.ones(n)
    if n % 2 == 0:
        real[(root + n // 2) % n] = 2.0
    # parent: the larger of the (one or two) neighbours one step closer
    par = np.empty(n, np.int64)
    for v in range(n):
        if v == root:
            par[v] = root
            continue
        cands = [w for w in ((v - 1) % n, (v + 1) % n) if dist[w] == dist[v] - 1]
        par[v] = max(cands)
    _all_checks(g, root, dist, par, real)


@pytest.mark.parametrize("n,root", [(2, 0), (6, 0), (6, 4), (65, 1)])
def test_star(n, root):
    g = _csr_from_pairs(n, [(0, i) for i in range(1, n)])
    dist = np.full(n, 2 if root != 0 else 1)
    dist[0] = 0 if root == 0 else 1
    dist[root] = 0
    par = np.zeros(n, np.int64)
    par[0] = root  # the centre hangs off a leaf root
    par[root] = root
    _all_checks(g, root, dist, par, np.ones(n))


@pytest.mark.parametrize("n,root", [(2, 0), (5, 3), (33, 32)])
def test_complete(n, root):
    g = _csr_from_pairs(n, list(itertools.combinations(range(n), 2)))
    dist = np.ones(n, np.int64)
    dist[root] = 0
    par = np.full(n, root)
    _all_checks(g, root, dist, par, np.ones(n))
    assert oracle.semiring_bfs(g, root, oracle.SELMAX).iterations == 2


@pytest.mark.parametrize("k,root", [(1, 0), (4, 0), (6, 37), (9, 300)])
def test_hypercube(k, root):
    n = 1 << k
    edges = [(v, v ^ (1 << b)) for v in range(n) for b in range(k) if v < v ^ (1 << b)]
    g = _csr_from_pairs(n, edges)
    v = np.arange(n)
    diff = v ^ root
    dist = np.array([bin(x).count("1") for x in diff])
    par = np.empty(n, np.int64)
    for u in range(n):
        D = u ^ root
        if D == 0:
            par[u] = root
            continue
        up = D & ~u  # bits the root has and u lacks: setting one moves closer and up
        par[u] = (u | (1 << (up.bit_length() - 1))) if up else (u & ~(D & -D))
    _all_checks(g, root, dist, par, dist.astype(np.float64) + (diff == 0))


@pytest.mark.parametrize("w,h,xr,yr", [(2, 2, 0, 0), (5, 3, 2, 1), (16, 9, 15, 0), (7, 11, 3, 10)])
def test_full_grid(w, h, xr, yr):
    gg = graphgen.grid(w, h, 0.0)
    g = oracle.csr_from_edgelist(gg)
    root = yr * w + xr
    ids = np.arange(w * h)
    x, y = ids % w, ids // w
    dist = np.abs(x - xr) + np.abs(y - yr)
    par = np.where(y < yr, ids + w,
                   np.where(x < xr, ids + 1,
                            np.where(x > xr, ids - 1,
                                     np.where(y > yr, ids - w, root))))
    real = np.where((x == xr) | (y == yr), 1.0, 2.0)
    _all_checks(g, root, dist, par, real)


def test_disconnected_and_isolated_root():
    g = _csr_from_pairs(6, [(0, 1), (1, 2), (4, 5)])
    _all_checks(g, 0, np.array([0, 1, 2, -1, -1, -1]), np.array([0, 0, 1, -1, -1, -1]),
                [1, 1, 1, 0, 0, 0])
    _all_checks(g, 3, np.array([-1, -1, -1, 0, -1, -1]), np.array([-1, -1, -1, 3, -1, -1]),
                [0, 0, 0, 1, 0, 0])
    assert oracle.semiring_bfs(g, 3, oracle.BOOLEAN).iterations == 1


# ------------------------------------------------------------- invariants

def _check_invariants(g, root, ex):
    d = ex.dist
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    a, b = rows, g.adj
    both = (d[a] >= 0) & (d[b] >= 0)
    assert np.all(np.abs(d[a][both] - d[b][both]) <= 1)          # edges span <= 1 level
    assert not np.any((d[a] >= 0) & (d[b] < 0))                  # reached set is closed
    assert d[root] == 0
    reached = np.flatnonzero(d > 0)
    p = ex.parent
    assert p[root] == root
    assert np.all(p[d < 0] == -1)
    assert np.all(d[p[reached]] == d[reached] - 1)               # parent one level up
    # parent is a neighbour, and no larger neighbour qualifies
    for v in reached[:: max(1, len(reached) // 2000)]:
        nb = g.adj[g.rowptr[v]:g.rowptr[v + 1]]
        assert p[v] in nb
        up = nb[d[nb] == d[v] - 1]
        assert up.max() == p[v]
        assert ex.real_val[v] == float(len(up))


@pytest.mark.parametrize("kind", ["rmat", "er"])
def test_invariants_and_semiring_agreement_on_random_graphs(kind):
    if kind == "rmat":
        e = graphgen.rmat(12, 16, seed=1)
    else:
        e = graphgen.er(5000, 40000, seed=2)
    g = oracle.csr_from_edgelist(e)
    roots = graphgen.pick_roots(e, 5, seed=11)
    for root in roots:
        ex = oracle.expected(g, int(root))
        _check_invariants(g, int(root), ex)
        levels = np.bincount(ex.dist[ex.dist > 0]) if (ex.dist > 0).any() else np.zeros(1)
        for s in SEMIRINGS:
            r = oracle.semiring_bfs(g, int(root), s)
            np.testing.assert_array_equal(r.dist, ex.dist)
            assert r.iterations == ex.iterations
            np.testing.assert_array_equal(r.frontier_sizes[:-1], levels[1:])
            assert r.frontier_sizes[-1] == 0
            if s == oracle.SELMAX:
                np.testing.assert_array_equal(r.parent, ex.parent)
            if s == oracle.REAL:
                np.testing.assert_array_equal(r.real_val, ex.real_val)
        np.testing.assert_array_equal(oracle.bfs_omp(g, int(root)), ex.dist)


def test_iteration_cap_is_reported():
    g = _csr_from_pairs(10, [(i, i + 1) for i in range(9)])
    with pytest.raises(ValueError):
        oracle.semiring_bfs(g, 0, oracle.TROPICAL, max_iters=3)
