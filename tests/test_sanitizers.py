"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the SlimSell layout builder (paper_2010_09913_amd/csrc/layout.cpp), the
oracle (oracle/oracle.c) and the input generators (graphgen/graphgen.c) are
compiled with -fsanitize=address,undefined and run by tests/sanitize_main.cpp
on small seeded graphs, which checks every layout against the oracle's
canonical graph and every oracle formulation against its queue BFS.  Any
sanitizer report aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIP_INCLUDE = "/opt/rocm/include"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]


@pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None,
                    reason="needs gcc and g++")
@pytest.mark.skipif(not os.path.isdir(os.path.join(HIP_INCLUDE, "hip")),
                    reason="layout.cpp's header needs the HIP headers")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    objs = []
    for src in ("oracle/oracle.c", "graphgen/graphgen.c"):
        obj = tmp_path / (os.path.basename(src) + ".o")
        subprocess.run(["gcc", "-std=c11", "-fopenmp", *SAN, "-c", os.path.join(ROOT, src),
                        "-o", str(obj)], check=True)
        objs.append(str(obj))
    exe = tmp_path / "sanitize_main"
    subprocess.run(["g++", "-std=c++17", "-fopenmp", "-pthread", *SAN, "-D__HIP_PLATFORM_AMD__",
                    "-I" + HIP_INCLUDE,
                    os.path.join(ROOT, "tests", "sanitize_main.cpp"),
                    os.path.join(ROOT, "paper_2010_09913_amd", "csrc", "layout.cpp"),
                    *objs, "-lm", "-o", str(exe)], check=True)
    env = dict(os.environ, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="abort_on_error=0:halt_on_error=1:detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    assert "0 failure(s)" in r.stderr
    assert r.stderr.count("\nok ") + r.stderr.startswith("ok ") == 5, r.stderr
