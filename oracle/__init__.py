"""ORACLE -- test infrastructure only.

Plain CPU statement of what SlimSell BFS computes (see ``oracle.c`` for the
definitions and the paper sections they follow).  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package.  It shares no code with the GPU path (``paper_2010_09913_amd``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

TROPICAL, REAL, BOOLEAN, SELMAX = 0, 1, 2, 3
SEMIRINGS = {"tropical": TROPICAL, "real": REAL, "boolean": BOOLEAN, "selmax": SELMAX}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, OpenMP only for oracle_bfs_omp)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", _SRC, "-o", tmp])
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
        f32p = ctypes.POINTER(ctypes.c_float)
        f64p = ctypes.POINTER(ctypes.c_double)
        lib.oracle_csr.argtypes = [i32p, i32p, ctypes.c_int64, ctypes.c_int32, i64p, i32p]
        lib.oracle_csr.restype = ctypes.c_int64
        lib.oracle_bfs.argtypes = [i64p, i32p, ctypes.c_int32, ctypes.c_int32, i32p]
        lib.oracle_bfs.restype = ctypes.c_int64
        lib.oracle_bfs_omp.argtypes = [i64p, i32p, ctypes.c_int32, ctypes.c_int32, i32p]
        lib.oracle_bfs_omp.restype = ctypes.c_int32
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int32
        lib.oracle_parents_max.argtypes = [i64p, i32p, ctypes.c_int32, ctypes.c_int32, i32p, i32p]
        lib.oracle_parents_max.restype = None
        lib.oracle_real_counts.argtypes = [i64p, i32p, ctypes.c_int32, ctypes.c_int32, i32p, f32p]
        lib.oracle_real_counts.restype = None
        lib.oracle_lneg.argtypes = [f64p, ctypes.c_int64, f64p]
        lib.oracle_lneg.restype = None
        lib.oracle_semiring_bfs.argtypes = [i64p, i32p, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_int32, i32p, i32p, f32p, i64p]
        lib.oracle_semiring_bfs.restype = ctypes.c_int32
        _lib = lib
    return _lib


def _p(a: np.ndarray | None, ct):
    if a is None:
        return ctypes.cast(None, ctypes.POINTER(ct))
    return a.ctypes.data_as(ctypes.POINTER(ct))


@dataclass
class CSR:
    """Canonical simple undirected graph (sorted, deduplicated rows)."""
    n: int
    rowptr: np.ndarray  # int64[n+1]
    adj: np.ndarray     # int32[E]

    @property
    def entries(self) -> int:
        return int(self.rowptr[-1])

    @property
    def degree(self) -> np.ndarray:
        return np.diff(self.rowptr)


def csr(n: int, src: np.ndarray, dst: np.ndarray) -> CSR:
    src = np.ascontiguousarray(src, np.int32)
    dst = np.ascontiguousarray(dst, np.int32)
    rowptr = np.empty(n + 1, np.int64)
    adj = np.empty(max(2 * src.shape[0], 1), np.int32)
    e = _load().oracle_csr(_p(src, ctypes.c_int32), _p(dst, ctypes.c_int32), src.shape[0], n,
                           _p(rowptr, ctypes.c_int64), _p(adj, ctypes.c_int32))
    if e < 0:
        raise ValueError(f"oracle_csr failed ({e})")
    return CSR(n, rowptr, adj[:e].copy())


def csr_from_edgelist(g) -> CSR:
    return csr(g.n, g.src, g.dst)


def bfs(g: CSR, root: int) -> np.ndarray:
    dist = np.empty(g.n, np.int32)
    r = _load().oracle_bfs(_p(g.rowptr, ctypes.c_int64), _p(g.adj, ctypes.c_int32), g.n, root,
                           _p(dist, ctypes.c_int32))
    if r < 0:
        raise ValueError("oracle_bfs failed")
    return dist


def threads() -> int:
    """Threads the OpenMP BFS uses."""
    return int(_load().oracle_threads())


def bfs_omp(g: CSR, root: int) -> np.ndarray:
    dist = np.empty(g.n, np.int32)
    r = _load().oracle_bfs_omp(_p(g.rowptr, ctypes.c_int64), _p(g.adj, ctypes.c_int32), g.n,
                               root, _p(dist, ctypes.c_int32))
    if r < 0:
        raise ValueError("oracle_bfs_omp failed")
    return dist


def parents_max(g: CSR, root: int, dist: np.ndarray) -> np.ndarray:
    par = np.empty(g.n, np.int32)
    _load().oracle_parents_max(_p(g.rowptr, ctypes.c_int64), _p(g.adj, ctypes.c_int32), g.n, root,
                               _p(np.ascontiguousarray(dist, np.int32), ctypes.c_int32),
                               _p(par, ctypes.c_int32))
    return par


def real_counts(g: CSR, root: int, dist: np.ndarray) -> np.ndarray:
    out = np.empty(g.n, np.float32)
    _load().oracle_real_counts(_p(g.rowptr, ctypes.c_int64), _p(g.adj, ctypes.c_int32), g.n, root,
                               _p(np.ascontiguousarray(dist, np.int32), ctypes.c_int32),
                               _p(out, ctypes.c_float))
    return out


def lneg(x) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float64)
    out = np.empty_like(x)
    _load().oracle_lneg(_p(x, ctypes.c_double), x.shape[0], _p(out, ctypes.c_double))
    return out


@dataclass
class SemiringResult:
    dist: np.ndarray
    parent: np.ndarray | None
    real_val: np.ndarray | None
    iterations: int
    frontier_sizes: np.ndarray


def semiring_bfs(g: CSR, root: int, semiring: int, max_iters: int = 0) -> SemiringResult:
    """Literal dense-vector stepping of one semiring formulation."""
    dist = np.empty(g.n, np.int32)
    par = np.empty(g.n, np.int32) if semiring == SELMAX else None
    rv = np.empty(g.n, np.float32) if semiring == REAL else None
    cap = max_iters if max_iters > 0 else g.n + 1
    fs = np.zeros(cap, np.int64)
    k = _load().oracle_semiring_bfs(_p(g.rowptr, ctypes.c_int64), _p(g.adj, ctypes.c_int32), g.n,
                                    root, semiring, cap, _p(dist, ctypes.c_int32),
                                    _p(par, ctypes.c_int32), _p(rv, ctypes.c_float),
                                    _p(fs, ctypes.c_int64))
    if k < 0:
        raise ValueError(f"oracle_semiring_bfs failed ({k})")
    return SemiringResult(dist, par, rv, int(k), fs[:k].copy())


@dataclass
class Expected:
    """What every GPU form must reproduce for one root (original vertex IDs)."""
    dist: np.ndarray
    parent: np.ndarray
    real_val: np.ndarray
    iterations: int


def expected(g: CSR, root: int) -> Expected:
    """Distances, max-ID parents, real values and the iteration count
    (eccentricity + 1) from the queue BFS plus the DP transformation."""
    d = bfs(g, root)
    par = parents_max(g, root, d)
    rv = real_counts(g, root, d)
    iters = int(d.max()) + 1
    return Expected(d, par, rv, iters)


def component_edges(g: CSR, dist: np.ndarray) -> int:
    """Undirected edges with both endpoints reached (the Graph500 TEPS numerator)."""
    reached = dist >= 0
    deg = g.degree
    return int(deg[reached].sum() // 2)
