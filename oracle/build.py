"""Compile the oracle (plain C, FP64, no FMA contraction, OpenMP static).

Test infrastructure only: the checker is built here, never used by the
product path.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libryo.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", os.path.join(HERE, "ryo.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    src = os.path.join(HERE, "ryo.c")
    hdr = os.path.join(HERE, "ryo.h")
    if (not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(src)
            or os.path.getmtime(LIB) < os.path.getmtime(hdr)):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
