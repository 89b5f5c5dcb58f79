"""Compile the oracle (plain C, FP64, no FMA contraction, OpenMP static).

Test infrastructure only: the checker is built here, never used by the
product path.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libryo.so")
SOURCES = ["ryo.c", "poisson.c"]
HEADERS = ["ryo.h", "poisson.h"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", LIB + ".tmp"] + [os.path.join(HERE, f) for f in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB) or any(os.path.getmtime(LIB) < os.path.getmtime(os.path.join(HERE, f))
                                      for f in SOURCES + HEADERS):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
