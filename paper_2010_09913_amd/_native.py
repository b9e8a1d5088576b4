"""ctypes declarations of libslimsell.so (the C ABI in include/slimsell.h).

The library is loaded from this package directory only; there is no fallback:
if it is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslimsell.so")

c_i32p = ctypes.POINTER(ctypes.c_int32)
c_i64p = ctypes.POINTER(ctypes.c_int64)
c_f32p = ctypes.POINTER(ctypes.c_float)

SS_OK, SS_EINVAL, SS_ENOMEM, SS_EHIP, SS_EUNSUP, SS_EITER = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "SS_OK", -1: "SS_EINVAL", -2: "SS_ENOMEM", -3: "SS_EHIP", -4: "SS_EUNSUP",
                -5: "SS_EITER"}

# Every symbol include/slimsell.h declares (checked by the tests).
EXPORTS = [
    "slimsell_layout_build", "slimsell_layout_view", "slimsell_layout_free",
    "slimsell_build", "slimsell_build_from_layout", "slimsell_graph_info",
    "slimsell_graph_degrees", "slimsell_tune_set", "slimsell_tune_get", "slimsell_free",
    "slimsell_bfs", "slimsell_sync", "slimsell_last_error", "slimsell_version",
    "slimsell_build_multi", "slimsell_graph_parts", "slimsell_bfs_batch", "slimsell_autotune",
    "slimsell_sched_load", "slimsell_sched_clear", "slimsell_sched_log", "slimsell_sched_grad",
    "slimsell_sched_forward", "slimsell_sched_train", "slimsell_dp_parents",
    "slimsell_bfs_noalloc",
]
SCHED_PARAMS, SCHED_FEATURES, SCHED_VARIANTS = 1412, 6, 4


class LayoutView(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("n_pad", ctypes.c_int32), ("C", ctypes.c_int32),
        ("sigma", ctypes.c_int32), ("n_chunks", ctypes.c_int64), ("entries", ctypes.c_int64),
        ("cells", ctypes.c_int64), ("max_cl", ctypes.c_int32), ("pad0", ctypes.c_int32),
        ("col", c_i32p), ("cs", c_i64p), ("cl", c_i32p), ("v", c_i32p), ("perm", c_i32p),
        ("degree", c_i32p),
    ]


class LevelStats(ctypes.Structure):
    _fields_ = [
        ("discovered", ctypes.c_int64), ("frontier_edges", ctypes.c_int64),
        ("active_chunks", ctypes.c_int64), ("active_cells", ctypes.c_int64),
        ("max_active_cl", ctypes.c_int64), ("ms", ctypes.c_float), ("variant", ctypes.c_int32),
    ]


class RunStats(ctypes.Structure):
    _fields_ = [
        ("iterations", ctypes.c_int32), ("launches", ctypes.c_int32),
        ("kernel_ms", ctypes.c_float), ("bfs_ms", ctypes.c_float),
        ("dp_ms", ctypes.c_float), ("pad0", ctypes.c_int32),
        ("dp_chunks", ctypes.c_int64), ("dp_cells", ctypes.c_int64),
    ]


class Tune(ctypes.Structure):
    _fields_ = [
        ("split_len", ctypes.c_int32), ("waves_per_group", ctypes.c_int32),
        ("unroll", ctypes.c_int32), ("max_groups", ctypes.c_int32),
        ("pack_cols", ctypes.c_int32), ("lds_kib", ctypes.c_int32),
    ]


class AutotuneOpts(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_uint32), ("semiring", ctypes.c_int32), ("batched", ctypes.c_int32),
        ("num_roots", ctypes.c_int32), ("roots", c_i32p), ("repeats", ctypes.c_int32),
        ("force", ctypes.c_int32), ("stream", ctypes.c_void_p),
    ]


class AutotuneResult(ctypes.Structure):
    _fields_ = [
        ("best", Tune), ("best_ms", ctypes.c_float), ("before_ms", ctypes.c_float),
        ("evaluated", ctypes.c_int32), ("from_cache", ctypes.c_int32),
    ]


SS_STATS_TIME = 1
SS_STATS_COUNTERS = 2
SS_RUN_PERSISTENT = 4
SS_SELL_VAL = 8
SS_STATS_TIME_BFS = 16
SS_NO_SUMMARY = 32
SS_SCHED_LAZY = 64


class BfsOpts(ctypes.Structure):
    _fields_ = [
        ("size", ctypes.c_uint32), ("slimwork", ctypes.c_int32), ("split_len", ctypes.c_int32),
        ("waves_per_group", ctypes.c_int32), ("schedule", ctypes.c_int32),
        ("max_levels", ctypes.c_int32), ("stream", ctypes.c_void_p),
        ("iterations_out", c_i32p), ("flags", ctypes.c_int32), ("level_cap", ctypes.c_int32),
        ("level_stats_out", ctypes.POINTER(LevelStats)),
        ("run_stats_out", ctypes.POINTER(RunStats)),
    ]


_lib = None


def load() -> ctypes.CDLL:
    """Load libslimsell.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2010_09913_amd.build_native` "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    vpp = ctypes.POINTER(ctypes.c_void_p)
    lib.slimsell_layout_build.argtypes = [c_i32p, c_i32p, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, vpp]
    lib.slimsell_layout_view.argtypes = [vp, ctypes.POINTER(LayoutView)]
    lib.slimsell_layout_free.argtypes = [vp]
    lib.slimsell_layout_free.restype = None
    lib.slimsell_build.argtypes = [c_i32p, c_i32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, vp, vpp]
    lib.slimsell_build_from_layout.argtypes = [vp, vp, vpp]
    lib.slimsell_graph_info.argtypes = [vp, c_i64p, c_i64p, c_i64p, c_i64p, c_i64p]
    lib.slimsell_graph_degrees.argtypes = [vp, c_i32p]
    lib.slimsell_tune_set.argtypes = [vp, ctypes.POINTER(Tune)]
    lib.slimsell_tune_get.argtypes = [vp, ctypes.POINTER(Tune)]
    lib.slimsell_free.argtypes = [vp]
    lib.slimsell_free.restype = None
    lib.slimsell_bfs.argtypes = [vp, c_i32p, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.POINTER(BfsOpts), vp, vp, vp]
    lib.slimsell_bfs_noalloc.argtypes = [vp, c_i32p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.POINTER(BfsOpts), vp, vp, vp]
    lib.slimsell_sync.argtypes = [vp]
    lib.slimsell_build_multi.argtypes = [ctypes.c_int32, c_i64p, c_i32p, c_i32p, c_i32p,
                                         ctypes.c_int32, ctypes.c_int32, vp, vpp]
    lib.slimsell_graph_parts.argtypes = [vp, c_i32p, c_i64p, c_i64p]
    lib.slimsell_bfs_batch.argtypes = [vp, c_i32p, ctypes.c_int32, ctypes.POINTER(BfsOpts), vp]
    lib.slimsell_autotune.argtypes = [vp, ctypes.POINTER(AutotuneOpts),
                                      ctypes.POINTER(AutotuneResult)]
    lib.slimsell_sched_load.argtypes = [c_f32p, ctypes.c_int64]
    lib.slimsell_sched_clear.argtypes = []
    lib.slimsell_sched_log.argtypes = [vp, c_f32p, ctypes.c_int32, c_i32p]
    lib.slimsell_sched_grad.argtypes = [c_f32p, c_f32p, c_f32p, ctypes.c_int64, c_f32p, c_f32p,
                                        vp]
    lib.slimsell_sched_forward.argtypes = [c_f32p, c_f32p, ctypes.c_int64, c_f32p, vp]
    lib.slimsell_sched_train.argtypes = [c_f32p, c_f32p, ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_float, ctypes.c_uint64, c_f32p, c_f32p, c_f32p,
                                         vp]
    lib.slimsell_dp_parents.argtypes = [vp, vp, ctypes.c_int32, vp, vp]
    lib.slimsell_last_error.argtypes = []
    lib.slimsell_last_error.restype = ctypes.c_char_p
    lib.slimsell_version.argtypes = []
    lib.slimsell_version.restype = ctypes.c_char_p
    for name in ("slimsell_layout_build", "slimsell_layout_view", "slimsell_build",
                 "slimsell_build_from_layout", "slimsell_graph_info",
                 "slimsell_graph_degrees", "slimsell_tune_set", "slimsell_tune_get",
                 "slimsell_bfs", "slimsell_sync", "slimsell_build_multi",
                 "slimsell_graph_parts", "slimsell_bfs_batch", "slimsell_autotune",
                 "slimsell_sched_load", "slimsell_sched_clear", "slimsell_sched_log",
                 "slimsell_sched_grad", "slimsell_sched_forward", "slimsell_sched_train",
                 "slimsell_dp_parents", "slimsell_bfs_noalloc"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class SlimSellError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(rc: int) -> None:
    if rc != SS_OK:
        msg = load().slimsell_last_error()
        raise SlimSellError(rc, msg.decode() if msg else "")
