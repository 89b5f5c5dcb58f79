"""The debug build of the library (device index bounds checks, see
ry_internal.h debug_in_bounds) runs the workloads' code paths clean: uniform
and AMR meshes, periodic and outflow, sides of 2 mod 4 cells, both tile
shapes and both precision forms, a regrid, the batched boxes.  One child
process (the library is chosen when the binding loads)."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_debug_build_runs_clean():
    lib = os.path.join(os.path.dirname(HERE), "paper_2411_14631_amd", "libry_debug.so")
    if not os.path.exists(lib):
        pytest.fail("libry_debug.so is missing: build it with __graft_entry__.build()")
    env = dict(os.environ, RY_DEBUG_LIB="1")
    r = subprocess.run([sys.executable, "-u", os.path.join(HERE, "debug_bounds_cases.py")], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.count("clean:") == 8, r.stdout
