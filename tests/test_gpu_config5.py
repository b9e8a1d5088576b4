"""GPU parity at the full sizes of the learned-schedule workload: R-MAT scale
24 (edge factor 16, seed 1) and the 4096 x 4096 grid with 5 % of its edges
removed (seed 5), sel-max semiring, sigma = n, roots drawn with seed 1005.

The grid's BFS runs about 5,000 levels, so every per-level ring of the
scheduled path (variants, queue lengths, counters, reports; 1,024 entries
each) wraps several times.  Distances and parents are compared element by
element with the oracle's queue BFS and max-ID parent pass, and the iteration
count with eccentricity + 1, under no schedule, the learned schedule (the
committed model), the fixed heuristic and forced push, each launched per
level and as one persistent launch.

The oracle of R-MAT scale 24 takes minutes on the CPU, so its stages are
tests of their own (each prints its progress when it ends).
"""
import os
import sys
import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

MODES = ["none", "learned", "heuristic", "push"]
_C = {}


@pytest.fixture(scope="module")
def ss():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2010_09913_amd as mod
    return mod


def note(*a):
    print(*a, file=sys.stderr, flush=True)


def _edges(name):
    key = ("e", name)
    if key not in _C:
        if name == "rmat24":
            _C[key] = graphgen.rmat(24, 16, seed=1)
        else:
            _C[key] = graphgen.grid(4096, 4096, 0.05, seed=5)
    return _C[key]


def _roots(name):
    return graphgen.pick_roots(_edges(name), 2 if name == "rmat24" else 1, seed=1005)


def _expected(name):
    """Oracle distances, max-ID parents and iteration counts of the roots."""
    key = ("x", name)
    if key not in _C:
        t = time.perf_counter()
        g = oracle.csr_from_edgelist(_edges(name))
        out = []
        for r in _roots(name):
            d = oracle.bfs(g, int(r))
            out.append((int(r), d, oracle.parents_max(g, int(r), d), int(d.max()) + 1))
        del g
        _C[key] = out
        note(f"oracle {name}: {time.perf_counter() - t:.1f}s")
    return _C[key]


def _graph(ss, name):
    key = ("G", name)
    if key not in _C:
        t = time.perf_counter()
        _C[key] = ss.Graph.from_edgelist(_edges(name), sigma=0)
        note(f"device graph {name}: {time.perf_counter() - t:.1f}s")
    return _C[key]


def _model(ss):
    from paper_2010_09913_amd import scheduler
    path = scheduler.DEFAULT_MODEL
    assert os.path.exists(path), "the committed scheduler model is missing"
    return np.load(path)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["rmat24", "grid4096"])
def test_oracle_of_the_full_size_inputs(name):
    ex = _expected(name)
    for r, d, p, it in ex:
        assert d[r] == 0 and p[r] == r
        # the grid is connected after the cut in all but a few vertices and
        # has a diameter in the thousands; R-MAT's is small
        assert (it > 1000) if name == "grid4096" else (3 <= it <= 20)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["rmat24", "grid4096"])
def test_device_graph_of_the_full_size_inputs(ss, name):
    G = _graph(ss, name)
    e = _edges(name)
    assert G.info()["n"] == e.n


@pytest.mark.timeout(600)
@pytest.mark.parametrize("persistent", [False, True], ids=["per-level", "persistent"])
@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("name", ["rmat24", "grid4096"])
def test_schedules_match_the_oracle_at_full_size(ss, name, mode, persistent):
    import torch
    G = _graph(ss, name)
    ex = _expected(name)
    if mode == "learned":
        ss.sched_load(_model(ss))
    try:
        for r, d, p, it in ex:
            note(name, mode, "persistent" if persistent else "per-level", "root", r)
            res = G.bfs([r], "selmax", schedule=mode, persistent=persistent,
                        level_cap=it + 2 if mode != "none" else 0, counters=False)
            torch.cuda.synchronize()
            np.testing.assert_array_equal(res.dist[0].cpu().numpy(), d,
                                          err_msg=f"{name} {mode} root {r} dist")
            np.testing.assert_array_equal(res.parent[0].cpu().numpy(), p,
                                          err_msg=f"{name} {mode} root {r} parent")
            assert int(res.iterations[0]) == it
            if mode != "none":
                var = res.levels["variant"][0][:it]
                assert np.all((var >= 0) & (var < 4)), var
                if mode == "push":
                    assert np.all(var == 3)
                log = G.sched_log()
                assert log.shape[0] == it
                np.testing.assert_array_equal(log[:, 11], np.arange(1, it + 1))
    finally:
        ss.sched_clear()


@pytest.mark.timeout(600)
def test_full_size_inputs_release(ss):
    for key in [k for k in _C if k[0] == "G"]:
        _C.pop(key).close()
    _C.clear()
