"""The ctypes mirrors in the binding have the layout the C header gives
(compiled here with gcc), so every field crosses the boundary intact."""
import ctypes
import os
import subprocess

import pytest

from paper_2010_09913_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = {
    "ss_bfs_opts": _native.BfsOpts,
    "ss_level_stats": _native.LevelStats,
    "ss_run_stats": _native.RunStats,
    "ss_tune": _native.Tune,
    "ss_layout_view": _native.LayoutView,
    "ss_autotune_opts": _native.AutotuneOpts,
    "ss_autotune_result": _native.AutotuneResult,
}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    d = tmp_path_factory.mktemp("abi")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "slimsell.h"', 'int main(void) {']
    for name, cls in STRUCTS.items():
        lines.append(f'  printf("sizeof {name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines.append(f'  printf("params %d %d %d\\n", SS_SCHED_PARAMS, SS_SCHED_FEATURES, SS_SCHED_VARIANTS);')
    lines.append('  return 0; }')
    src = d / "abi.c"
    src.write_text("\n".join(lines))
    exe = d / "abi"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                           str(exe)])
    out = subprocess.check_output([str(exe)], text=True)
    table = {}
    for line in out.splitlines():
        parts = line.split()
        table[tuple(parts[:-1])] = int(parts[-1])
    return table


@pytest.mark.parametrize("name", list(STRUCTS))
def test_struct_layout_matches_header(c_layout, name):
    cls = STRUCTS[name]
    assert ctypes.sizeof(cls) == c_layout[("sizeof", name)]
    for f, _ in cls._fields_:
        assert getattr(cls, f).offset == c_layout[(name, f)], (name, f)


def test_scheduler_constants(c_layout):
    assert c_layout[("params", "1412", "6")] == 4
    assert (_native.SCHED_PARAMS, _native.SCHED_FEATURES, _native.SCHED_VARIANTS) == (1412, 6, 4)
