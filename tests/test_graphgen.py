"""Seeded input generators: determinism, sizes and the shape of the inputs."""
import numpy as np

import graphgen


def test_rmat_is_deterministic_and_seeded():
    a = graphgen.rmat(10, 16, seed=1)
    b = graphgen.rmat(10, 16, seed=1)
    c = graphgen.rmat(10, 16, seed=2)
    assert a.m == 16 * 1024 and a.n == 1024
    np.testing.assert_array_equal(a.src, b.src)
    np.testing.assert_array_equal(a.dst, b.dst)
    assert not np.array_equal(a.src, c.src)
    assert a.src.min() >= 0 and a.src.max() < a.n and a.dst.max() < a.n


def test_rmat_degree_is_skewed_and_er_is_not():
    r = graphgen.rmat(14, 16, seed=1)
    e = graphgen.er(1 << 14, 16 << 14, seed=2)
    dr = np.bincount(np.concatenate([r.src, r.dst]), minlength=r.n)
    de = np.bincount(np.concatenate([e.src, e.dst]), minlength=e.n)
    assert dr.max() > 20 * dr.mean()          # power-law hubs
    assert de.max() < 3 * de.mean()           # uniform degrees
    assert abs(de.mean() - 32) < 1e-9


def test_grid_removes_exactly_the_requested_edges():
    full = graphgen.grid(64, 64, 0.0)
    cut = graphgen.grid(64, 64, 0.05, seed=5)
    e = 2 * 63 * 64
    assert full.m == e
    assert cut.m == e - int(np.floor(0.05 * e + 0.5))
    keys_full = set(zip(full.src.tolist(), full.dst.tolist()))
    keys_cut = set(zip(cut.src.tolist(), cut.dst.tolist()))
    assert keys_cut <= keys_full
    assert abs(cut.src - cut.dst).max() in (1, 64)


def test_roots_are_distinct_nonisolated_and_seeded():
    g = graphgen.rmat(12, 16, seed=1)
    r1 = graphgen.pick_roots(g, 64, seed=1003)
    r2 = graphgen.pick_roots(g, 64, seed=1003)
    np.testing.assert_array_equal(r1, r2)
    assert len(set(r1.tolist())) == 64
    deg = np.bincount(np.concatenate([g.src[g.src != g.dst], g.dst[g.src != g.dst]]), minlength=g.n)
    assert np.all(deg[r1] > 0)


def test_er_set_params_follow_the_stated_ranges():
    n, m, s = graphgen.er_set_params(256, seed=3)
    assert n.min() >= 2 ** 10 and n.max() <= 2 ** 18
    rho = 2 * m / n
    assert rho.min() >= 8 - 1e-2 and rho.max() <= 64 + 1e-2
    assert len(set(s.tolist())) == 256
