"""Seeded synthetic graph inputs (R-MAT, Erdos-Renyi, grid) and root draws.

The generators stand in for the paper's Kronecker and Erdos-Renyi inputs
(Section IV, "Selection of Benchmarks and Parameters"; Table "graphs").  They
return raw (src, dst) tuples as int32 numpy arrays; self-loops and duplicates
are kept and each consumer canonicalises the graph itself.

This package holds no BFS arithmetic.  It is the only code that the oracle and
the GPU path share.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None

RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = True) -> str:
    """Compile libgraphgen.so in-tree with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c11", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                ctypes.c_double, ctypes.c_uint64, i32p, i32p]
        lib.gg_rmat.restype = ctypes.c_int
        lib.gg_er.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, i32p, i32p]
        lib.gg_er.restype = ctypes.c_int
        lib.gg_grid_edges.argtypes = [ctypes.c_int32, ctypes.c_int32]
        lib.gg_grid_edges.restype = ctypes.c_int64
        lib.gg_grid.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                i32p, i32p]
        lib.gg_grid.restype = ctypes.c_int64
        lib.gg_er_set_params.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                         i64p, i64p, u64p]
        lib.gg_er_set_params.restype = ctypes.c_int
        lib.gg_pick_roots.argtypes = [i32p, i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_uint64, i32p]
        lib.gg_pick_roots.restype = ctypes.c_int32
        lib.gg_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        lib.gg_draw.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


@dataclass
class EdgeList:
    """Raw tuples of an undirected graph on vertices [0, n)."""
    n: int
    src: np.ndarray
    dst: np.ndarray
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def rmat(scale: int, edge_factor: int = 16, seed: int = 1, abc=RMAT_ABC) -> EdgeList:
    """R-MAT with 2^scale vertices and edge_factor * 2^scale tuples."""
    n = 1 << scale
    m = edge_factor * n
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    rc = _load().gg_rmat(scale, m, abc[0], abc[1], abc[2], seed, _p32(src), _p32(dst))
    if rc != 0:
        raise RuntimeError(f"gg_rmat failed ({rc})")
    return EdgeList(n, src, dst, f"rmat-s{scale}-ef{edge_factor}-seed{seed}")


def er(n: int, m: int, seed: int) -> EdgeList:
    """Erdos-Renyi G(n, M) with m uniform tuples."""
    src = np.empty(m, np.int32)
    dst = np.empty(m, np.int32)
    rc = _load().gg_er(n, m, seed, _p32(src), _p32(dst))
    if rc != 0:
        raise RuntimeError(f"gg_er failed ({rc})")
    return EdgeList(n, src, dst, f"er-n{n}-m{m}-seed{seed}")


def grid(w: int, h: int, remove_frac: float = 0.0, seed: int = 5) -> EdgeList:
    """W x H 4-neighbour grid with round(remove_frac * edges) edges removed."""
    lib = _load()
    e = lib.gg_grid_edges(w, h)
    remove = int(np.floor(remove_frac * e + 0.5))
    src = np.empty(e, np.int32)
    dst = np.empty(e, np.int32)
    got = lib.gg_grid(w, h, remove, seed, _p32(src), _p32(dst))
    if got < 0:
        raise RuntimeError(f"gg_grid failed ({got})")
    return EdgeList(w * h, src[:got].copy(), dst[:got].copy(), f"grid-{w}x{h}-rm{remove}-seed{seed}")


def er_set_params(count: int, seed: int, lo_log2=10.0, hi_log2=18.0, rho_lo=8.0, rho_hi=64.0):
    """(n_i, m_i, sub_seed_i) of a set of ER graphs with log-uniform sizes."""
    n = np.empty(count, np.int64)
    m = np.empty(count, np.int64)
    s = np.empty(count, np.uint64)
    rc = _load().gg_er_set_params(
        count, lo_log2, hi_log2, rho_lo, rho_hi, seed,
        n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        m.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
        s.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise RuntimeError("gg_er_set_params failed")
    return n, m, s


def er_set(count: int, seed: int, **kw) -> list[EdgeList]:
    n, m, s = er_set_params(count, seed, **kw)
    return [er(int(n[i]), int(m[i]), int(s[i])) for i in range(count)]


def pick_roots(g: EdgeList, k: int, seed: int) -> np.ndarray:
    """Up to k distinct roots drawn uniformly from the nonzero-degree vertices."""
    out = np.empty(max(k, 1), np.int32)
    got = _load().gg_pick_roots(_p32(g.src), _p32(g.dst), g.m, g.n, k, seed, _p32(out))
    if got < 0:
        raise RuntimeError("gg_pick_roots failed")
    return out[:got].copy()


def draw(seed: int, stream: int, ctr: int) -> int:
    """The raw 64-bit counter-based draw (exposed for tests)."""
    return int(_load().gg_draw(seed, stream, ctr))
