"""MI355X SlimSell BFS: Python binding of libslimsell.so.

Argument marshalling only.  The layout build runs in the library's host C++
code and every BFS step runs in its HIP kernels; PyTorch provides device
memory and streams.  Names follow the C ABI in include/slimsell.h.

Paper: Besta et al., "SlimSell: A Vectorizable Graph Representation for
Breadth-First Search" (arXiv 2010.09913).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _native
from ._native import BfsOpts, LayoutView, SlimSellError, check

TROPICAL, REAL, BOOLEAN, SELMAX = 0, 1, 2, 3
SEMIRINGS = {"tropical": TROPICAL, "real": REAL, "boolean": BOOLEAN, "selmax": SELMAX}
CHUNK = 64

__all__ = ["Graph", "Layout", "layout_build", "SlimSellError", "SEMIRINGS", "TROPICAL", "REAL",
           "BOOLEAN", "SELMAX", "version"]


def _semiring(s) -> int:
    if isinstance(s, str):
        return SEMIRINGS[s]
    return int(s)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _p32(a: np.ndarray):
    return a.ctypes.data_as(_native.c_i32p)


def version() -> str:
    return _native.load().slimsell_version().decode()


@dataclass
class Layout:
    """Host copy of a SlimSell layout (see ss_layout_view in slimsell.h)."""
    n: int
    n_pad: int
    sigma: int
    n_chunks: int
    entries: int
    cells: int
    max_cl: int
    col: np.ndarray
    cs: np.ndarray
    cl: np.ndarray
    v: np.ndarray
    perm: np.ndarray
    degree: np.ndarray

    @property
    def padding(self) -> int:
        return self.cells - self.entries


def layout_build(src, dst, n: int, sigma: int = 0, C: int = CHUNK,
                 arrays: bool = True) -> Layout:
    """Build the SlimSell layout on the host and copy it out (no device needed);
    arrays=False returns the sizes only (empty arrays)."""
    lib = _native.load()
    src = _i32(src)
    dst = _i32(dst)
    h = ctypes.c_void_p()
    check(lib.slimsell_layout_build(_p32(src), _p32(dst), src.shape[0], n, C, sigma,
                                    ctypes.byref(h)))
    try:
        v = LayoutView()
        check(lib.slimsell_layout_view(h, ctypes.byref(v)))

        def arr(ptr, count, dt):
            if count == 0 or not arrays:
                return np.zeros(0, dt)
            return np.ctypeslib.as_array(ptr, shape=(count,)).astype(dt, copy=True)

        return Layout(v.n, v.n_pad, v.sigma, v.n_chunks, v.entries, v.cells, v.max_cl,
                      arr(v.col, v.cells, np.int32), arr(v.cs, v.n_chunks + 1, np.int64),
                      arr(v.cl, v.n_chunks, np.int32), arr(v.v, v.n_pad, np.int32),
                      arr(v.perm, v.n, np.int32), arr(v.degree, v.n_pad, np.int32))
    finally:
        lib.slimsell_layout_free(h)


LEVEL_FIELDS = ("discovered", "frontier_edges", "active_chunks", "active_cells",
                "max_active_cl", "ms", "variant")
_LEVEL_DTYPE = np.dtype([("discovered", "<i8"), ("frontier_edges", "<i8"),
                         ("active_chunks", "<i8"), ("active_cells", "<i8"),
                         ("max_active_cl", "<i8"), ("ms", "<f4"), ("variant", "<i4")])
_RUN_DTYPE = np.dtype([("iterations", "<i4"), ("launches", "<i4"), ("kernel_ms", "<f4"),
                       ("bfs_ms", "<f4"), ("dp_ms", "<f4"), ("pad0", "<i4"),
                       ("dp_chunks", "<i8"), ("dp_cells", "<i8")])


def _records(buf, dtype, shape):
    """Copy a ctypes array of records into a dict of numpy arrays."""
    arr = np.frombuffer(buf, dtype=dtype).reshape(shape)
    return {f: arr[f].copy() for f in dtype.names}
VARIANTS = ("pull", "pull-split256", "pull-split1024", "push")
SCHEDULES = {"none": 0, "learned": 1, "heuristic": 2, "pull": 3, "pull-split256": 4,
             "pull-split1024": 5, "push": 6}
RUN_FIELDS = ("iterations", "launches", "kernel_ms", "bfs_ms", "dp_ms", "dp_chunks", "dp_cells")


@dataclass
class BfsResult:
    dist: "object"             # torch int32 [num_roots, n] (device)
    parent: "object | None"    # torch int32 [num_roots, n] (sel-max, or any with dp=True)
    real_val: "object | None"  # torch float32 [num_roots, n] (real only)
    iterations: np.ndarray     # int32 [num_roots]
    levels: dict | None = None  # field -> array [num_roots, level_cap]
    runs: dict | None = None    # field -> array [num_roots]

    @property
    def frontier(self):
        """Vertices discovered per level of the first root (needs counters)."""
        return None if self.levels is None else self.levels["discovered"][0]


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


class Graph:
    """A SlimSell graph resident on the current HIP device."""

    def __init__(self, src, dst, n: int, sigma: int = 0, stream=None):
        lib = _native.load()
        src = _i32(src)
        dst = _i32(dst)
        self._h = ctypes.c_void_p()
        self.n = int(n)
        self.sigma = sigma
        st = ctypes.c_void_p() if stream is None else _stream_handle(stream)
        check(lib.slimsell_build(_p32(src), _p32(dst), src.shape[0], n, CHUNK, sigma, st,
                                 ctypes.byref(self._h)))

    @classmethod
    def from_edgelist(cls, g, sigma: int = 0, stream=None) -> "Graph":
        return cls(g.src, g.dst, g.n, sigma=sigma, stream=stream)

    @classmethod
    def from_many(cls, graphs, sigma: int = 0, stream=None) -> "Graph":
        """Disjoint union of several edge lists as one device graph
        (slimsell_build_multi); graph i's vertex v is union vertex voff_i + v."""
        lib = _native.load()
        offs = np.zeros(len(graphs) + 1, np.int64)
        offs[1:] = np.cumsum([g.m for g in graphs])
        src = _i32(np.concatenate([g.src for g in graphs])) if graphs else np.zeros(0, np.int32)
        dst = _i32(np.concatenate([g.dst for g in graphs])) if graphs else np.zeros(0, np.int32)
        ns = _i32([g.n for g in graphs])
        self = cls.__new__(cls)
        self._h = ctypes.c_void_p()
        self.n = int(ns.sum())
        self.sigma = sigma
        st = ctypes.c_void_p() if stream is None else _stream_handle(stream)
        check(lib.slimsell_build_multi(len(graphs), offs.ctypes.data_as(_native.c_i64p),
                                       _p32(src), _p32(dst), _p32(ns), CHUNK, sigma, st,
                                       ctypes.byref(self._h)))
        return self

    def parts(self) -> tuple[np.ndarray, np.ndarray]:
        """(vertices per graph, union-ID offset per graph)."""
        lib = _native.load()
        k = ctypes.c_int32()
        check(lib.slimsell_graph_parts(self._h, ctypes.byref(k), None, None))
        ns = np.zeros(k.value, np.int64)
        off = np.zeros(k.value, np.int64)
        check(lib.slimsell_graph_parts(self._h, ctypes.byref(k), ns.ctypes.data_as(_native.c_i64p),
                                       off.ctypes.data_as(_native.c_i64p)))
        return ns, off

    def info(self) -> dict:
        vals = [ctypes.c_int64() for _ in range(5)]
        check(_native.load().slimsell_graph_info(self._h, *[ctypes.byref(x) for x in vals]))
        n, entries, padding, chunks, max_cl = (x.value for x in vals)
        return dict(n=n, entries=entries, padding=padding, chunks=chunks, max_cl=max_cl,
                    cells=entries + padding)

    def degrees(self) -> np.ndarray:
        """Canonical degree of every vertex (original IDs)."""
        out = np.empty(self.n, np.int32)
        check(_native.load().slimsell_graph_degrees(self._h, _p32(out)))
        return out

    TUNE_FIELDS = ("split_len", "waves_per_group", "unroll", "max_groups", "pack_cols", "lds_kib")

    def get_tune(self) -> dict:
        t = _native.Tune()
        check(_native.load().slimsell_tune_get(self._h, ctypes.byref(t)))
        return {f: getattr(t, f) for f in self.TUNE_FIELDS}

    def set_tune(self, **kw) -> dict:
        """Update the graph's launch configuration (fields of ss_tune)."""
        cur = self.get_tune()
        for k, v in kw.items():
            if k not in cur:
                raise KeyError(k)
            cur[k] = int(v)
        t = _native.Tune(**cur)
        check(_native.load().slimsell_tune_set(self._h, ctypes.byref(t)))
        return cur

    def bfs(self, roots, semiring="selmax", *, slimwork: int = 2, split_len: int = -1,
            waves_per_group: int = 0, schedule: int = 0, max_levels: int = 0, stream=None,
            level_cap: int = 0, timing: bool = False, counters: bool = None,
            persistent: bool = False, want_parent: bool = True, want_real: bool = True,
            dp: bool = False, sell: bool = False, summary: bool = True, dist=None,
            parent=None, real_val=None, no_alloc: bool = False,
            sched_lazy: bool = False) -> BfsResult:
        """BFS from every root; outputs are device tensors in original vertex IDs.

        Sel-max returns parents (unless want_parent=False); dp=True gives the
        other semirings parents too, by the DP transformation after each BFS.
        sell=True runs the Sell-C-sigma comparator (a val array beside col).
        summary=False turns off the frontier-summary filter of the gathers.
        sched_lazy=True makes the learned schedule stage its model only for
        levels inside the model's domain (SS_SCHED_LAZY).
        level_cap > 0 records per-level statistics (fused counters unless
        counters=False); timing=True adds event timings per level and per root,
        timing="bfs" per root only.  no_alloc=True calls the allocation-free
        entry point (slimsell_bfs_noalloc: no statistics, schedule, persistent
        launch or comparator; pass preallocated outputs to allocate nothing).
        """
        import torch
        s = _semiring(semiring)
        roots = _i32(np.atleast_1d(roots))
        nr = roots.shape[0]
        dev = torch.device("cuda", torch.cuda.current_device())
        for t, dt in ((dist, torch.int32), (parent, torch.int32), (real_val, torch.float32)):
            if t is not None and (t.dtype != dt or not t.is_cuda or not t.is_contiguous()
                                  or t.numel() != nr * self.n):
                raise ValueError(f"output tensors must be contiguous {dt} on the device with "
                                 f"num_roots * n = {nr * self.n} elements")
        if dist is None:
            dist = torch.empty((nr, self.n), dtype=torch.int32, device=dev)
        if parent is None and ((want_parent and s == SELMAX) or dp):
            parent = torch.empty((nr, self.n), dtype=torch.int32, device=dev)
        if real_val is None and want_real and s == REAL:
            real_val = torch.empty((nr, self.n), dtype=torch.float32, device=dev)
        iters = np.zeros(max(nr, 1), np.int32)
        o = BfsOpts()
        o.size = ctypes.sizeof(BfsOpts)
        o.slimwork = int(slimwork)
        o.split_len = split_len
        o.waves_per_group = waves_per_group
        o.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
        o.max_levels = max_levels
        o.stream = _stream_handle(stream)
        o.iterations_out = iters.ctypes.data_as(_native.c_i32p)
        if counters is None:
            counters = level_cap > 0
        o.flags = (_native.SS_STATS_TIME_BFS if timing == "bfs" else
                   _native.SS_STATS_TIME if timing else 0) | (
            _native.SS_STATS_COUNTERS if counters else 0) | (
            _native.SS_RUN_PERSISTENT if persistent else 0) | (
            _native.SS_SELL_VAL if sell else 0) | (
            0 if summary else _native.SS_NO_SUMMARY) | (
            _native.SS_SCHED_LAZY if sched_lazy else 0)
        lvl = runs = None
        if level_cap > 0:
            lvl = (_native.LevelStats * (nr * level_cap))()
            o.level_cap = level_cap
            o.level_stats_out = lvl
        if timing or level_cap > 0:
            runs = (_native.RunStats * max(nr, 1))()
            o.run_stats_out = runs

        def ptr(t):
            return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p()

        fn = _native.load().slimsell_bfs_noalloc if no_alloc else _native.load().slimsell_bfs
        check(fn(self._h, _p32(roots), nr, s, ctypes.byref(o), ptr(dist), ptr(parent),
                 ptr(real_val)))
        levels = run_d = None
        if lvl is not None:
            levels = _records(lvl, _LEVEL_DTYPE, (nr, level_cap))
        if runs is not None:
            run_d = {f: v[:nr] for f, v in _records(runs, _RUN_DTYPE, (max(nr, 1),)).items()}
        return BfsResult(dist, parent, real_val, iters[:nr].copy(), levels, run_d)

    def dp_parents(self, dist, parent=None, stream=None):
        """Parents from BFS distances (DP transformation): dist is an int32
        device tensor of num_roots * n elements in original vertex order."""
        import torch
        if dist.dtype != torch.int32 or not dist.is_cuda or not dist.is_contiguous() or \
                dist.numel() % max(self.n, 1):
            raise ValueError("dist must be a contiguous int32 device tensor of num_roots * n")
        nr = dist.numel() // max(self.n, 1)
        if parent is None:
            parent = torch.empty_like(dist)
        elif parent.dtype != torch.int32 or not parent.is_cuda or not parent.is_contiguous() \
                or parent.numel() != dist.numel():
            raise ValueError("parent must match dist")
        check(_native.load().slimsell_dp_parents(self._h, ctypes.c_void_p(dist.data_ptr()), nr,
                                                 ctypes.c_void_p(parent.data_ptr()),
                                                 _stream_handle(stream)))
        return parent

    def bfs_batch(self, roots, *, slimwork: int = 2, max_levels: int = 0, stream=None,
                  level_cap: int = 0, timing: bool = False, counters: bool = None,
                  persistent: bool = False, summary: bool = True, dist=None):
        """Batched BFS (64-bit frontier masks).  roots: int array [num_graphs, rpg]
        (graph-local IDs, -1 = unused slot) or [rpg] for a single graph.  Returns
        (dist tensor, iterations, levels, runs); dist holds each graph's block
        [rpg][n_i] at offset rpg * voff_i."""
        import torch
        roots = _i32(np.atleast_2d(roots))
        ng, rpg = roots.shape
        dev = torch.device("cuda", torch.cuda.current_device())
        if dist is None:
            dist = torch.empty(rpg * self.n, dtype=torch.int32, device=dev)
        elif dist.dtype != torch.int32 or not dist.is_cuda or dist.numel() != rpg * self.n:
            raise ValueError("dist must be an int32 device tensor of rpg * n elements")
        iters = np.zeros(1, np.int32)
        o = BfsOpts()
        o.size = ctypes.sizeof(BfsOpts)
        o.slimwork = int(slimwork)
        o.split_len = -1
        o.max_levels = max_levels
        o.stream = _stream_handle(stream)
        o.iterations_out = iters.ctypes.data_as(_native.c_i32p)
        if counters is None:
            counters = level_cap > 0
        o.flags = (_native.SS_STATS_TIME if timing else 0) | (
            _native.SS_STATS_COUNTERS if counters else 0) | (
            _native.SS_RUN_PERSISTENT if persistent else 0) | (
            0 if summary else _native.SS_NO_SUMMARY)
        lvl = runs = None
        if level_cap > 0:
            lvl = (_native.LevelStats * level_cap)()
            o.level_cap = level_cap
            o.level_stats_out = lvl
        if timing or level_cap > 0:
            runs = (_native.RunStats * 1)()
            o.run_stats_out = runs
        check(_native.load().slimsell_bfs_batch(self._h, _p32(roots.reshape(-1)), rpg,
                                                ctypes.byref(o), ctypes.c_void_p(dist.data_ptr())))
        levels = run_d = None
        if lvl is not None:
            levels = _records(lvl, _LEVEL_DTYPE, (level_cap,))
        if runs is not None:
            run_d = {f: v[0].item() for f, v in _records(runs, _RUN_DTYPE, (1,)).items()}
        return dist, int(iters[0]), levels, run_d

    def autotune(self, roots, semiring="selmax", *, batched: bool = False, repeats: int = 3,
                 force: bool = False, stream=None) -> dict:
        """Time launch configurations on these roots and keep the fastest."""
        roots2 = _i32(np.atleast_2d(roots)) if batched else _i32(np.atleast_1d(roots))[None, :]
        roots = roots2.reshape(-1)
        o = _native.AutotuneOpts()
        o.size = ctypes.sizeof(_native.AutotuneOpts)
        o.semiring = _semiring(semiring)
        o.batched = 1 if batched else 0
        o.num_roots = int(roots2.shape[1])
        o.roots = _p32(roots)
        o.repeats = repeats
        o.force = 1 if force else 0
        o.stream = _stream_handle(stream)
        r = _native.AutotuneResult()
        check(_native.load().slimsell_autotune(self._h, ctypes.byref(o), ctypes.byref(r)))
        return dict(best={f: getattr(r.best, f) for f in self.TUNE_FIELDS}, best_ms=r.best_ms,
                    before_ms=r.before_ms, evaluated=r.evaluated, from_cache=bool(r.from_cache))

    def sched_log(self, cap: int = 65536) -> np.ndarray:
        """[levels, 12] record of the last scheduled run: features, scores,
        variant, level."""
        out = np.zeros((cap, 12), np.float32)
        got = ctypes.c_int32()
        check(_native.load().slimsell_sched_log(self._h, out.ctypes.data_as(_native.c_f32p), cap,
                                                ctypes.byref(got)))
        return out[:got.value]

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            _native.load().slimsell_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sync(stream=None) -> None:
    check(_native.load().slimsell_sync(_stream_handle(stream)))


# ------------------------------------------------------------ scheduler model

def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _fp(a):
    return a.ctypes.data_as(_native.c_f32p)


def sched_load(weights) -> None:
    """Install the process-wide scheduler model: 1412 float32 parameters,
    optionally followed by its training domain (tau, K, K x 6 features)."""
    w = _f32(weights).reshape(-1)
    check(_native.load().slimsell_sched_load(_fp(w), w.shape[0]))


def sched_clear() -> None:
    check(_native.load().slimsell_sched_clear())


def sched_forward(weights, x) -> np.ndarray:
    w, x = _f32(weights).reshape(-1), _f32(x).reshape(-1, _native.SCHED_FEATURES)
    out = np.zeros((x.shape[0], _native.SCHED_VARIANTS), np.float32)
    check(_native.load().slimsell_sched_forward(_fp(w), _fp(x), x.shape[0], _fp(out),
                                                _stream_handle(None)))
    return out


def sched_grad(weights, x, y):
    """(loss, gradient) of the MSE loss on the GPU."""
    w = _f32(weights).reshape(-1)
    x = _f32(x).reshape(-1, _native.SCHED_FEATURES)
    y = _f32(y).reshape(-1, _native.SCHED_VARIANTS)
    g = np.zeros(_native.SCHED_PARAMS, np.float32)
    loss = np.zeros(1, np.float32)
    check(_native.load().slimsell_sched_grad(_fp(w), _fp(x), _fp(y), x.shape[0], _fp(g),
                                             _fp(loss), _stream_handle(None)))
    return float(loss[0]), g


def sched_train(x, y, steps: int = 2000, lr: float = 3e-3, seed: int = 0, init=None):
    """Train on the GPU; returns (weights, per-step loss)."""
    x = _f32(x).reshape(-1, _native.SCHED_FEATURES)
    y = _f32(y).reshape(-1, _native.SCHED_VARIANTS)
    w = np.zeros(_native.SCHED_PARAMS, np.float32)
    losses = np.zeros(max(steps, 1), np.float32)
    ini = _fp(_f32(init).reshape(-1)) if init is not None else ctypes.cast(None, _native.c_f32p)
    check(_native.load().slimsell_sched_train(_fp(x), _fp(y), x.shape[0], steps, lr, seed, ini,
                                              _fp(w), _fp(losses), _stream_handle(None)))
    return w, losses[:steps]
