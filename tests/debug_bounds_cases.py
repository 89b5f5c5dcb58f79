"""Run by test_gpu_debug_bounds.py in a child process with RY_DEBUG_LIB=1:
the workloads' code paths on the debug build of the library, whose device
index checks turn an access outside its buffer into an error at the next
syncing call.  Exits 0 when every case ran clean."""
import dataclasses
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import workloads as W  # noqa: E402
from paper_2411_14631_amd import ry  # noqa: E402

import cases  # noqa: E402

SMALL = (1, 0, 4, 1, 1, 4)
BIG = (1, 0, 4, 1, 8, 8)
BIG4 = (1, 0, 4, 1, 4, 8)   # the 8^3-cell tile on 4 wavefronts (two cells per thread)


def outflow(p):
    return dataclasses.replace(p, bc=(W.BC_OUTFLOW,) * 6)


def main():
    assert ry.LIB_PATH.endswith("libry_debug.so"), ry.LIB_PATH
    probs = [W.random_smooth(32, seed=3, mach=1.2), outflow(W.random_smooth(30, seed=4, mach=1.2)),
             cases.amr_blob(), cases.amr_blob(bc=(W.BC_OUTFLOW,) * 6, centre=(0.1, 0.5, 0.5)),
             outflow(W.twolevel(36, 0.5)), W.twolevel(64, 0.70), W.zoom(level_min=5, level_max=8)]
    for p in probs:
        for t in (SMALL, BIG, BIG4):
            for prec in ("fp64", "mixed"):
                h = ry.Hydro(p, prec)
                h.set_tuning(*t)
                h.advance(3)
                if p.level_max > p.level_min and prec == "fp64":
                    h.regrid()
                    h.advance(2)
                h.totals()
                h.close()
        print("clean:", p.name, flush=True)
    boxes = [W.batch_box(50, 24, 1.0, 1.5), W.batch_box(51, 18, 0.7, 0.8), W.batch_box(52, 16, 1.2, 2.0)]
    for t in (SMALL, BIG, BIG4):
        bh = ry.BatchHydro(boxes)
        bh.set_tuning(*t)
        bh.run(4)
        bh.close()
    print("clean: batch", flush=True)


if __name__ == "__main__":
    main()
