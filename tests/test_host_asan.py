"""The host C++ level planner (csrc/plan.cpp) built with the address and undefined-behaviour
sanitizers and run over 2D and 3D grids by tests/host/plan_check.cpp, which checks the
partition of Sec. 2.2 level by level (every DOF in one group, independent cells, every stencil
coupling and every cell's fill inside a planned block, exact provenance, a single root group).
The planner includes no HIP header, so the plain host compiler builds it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2004_05566_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_planner_under_address_and_ub_sanitizers(tmp_path):
    exe = str(tmp_path / "plan_check")
    cmd = ["g++", "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-I" + CSRC,
           os.path.join(CSRC, "plan.cpp"), os.path.join(ROOT, "tests", "host", "plan_check.cpp"),
           "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "all plans ok" in r.stdout
    assert r.stdout.count("\nok ") + r.stdout.startswith("ok ") == 14
