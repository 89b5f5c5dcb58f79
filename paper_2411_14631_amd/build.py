"""Build the HIP library (gfx950) in-tree: paper_2411_14631_amd/libry.so, and
its debug build libry_debug.so (-DRY_DEBUG: device index bounds checks that
latch an error instead of accessing out of bounds).

All sources go through hipcc.  Host code is compiled without floating-point
contraction (the refinement map must be a pure function of the input
bytes); the kernels opt into contraction locally.  Packed FP32 instructions
are disabled for all device code.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libry.so")
LIB_DEBUG = os.path.join(HERE, "libry_debug.so")
SOURCES = ["mesh.cpp", "api.cpp", "kernels.hip", "hydro.hip", "poisson.hip", "regrid.hip", "noalloc.hip"]
# per-source options: the hydro-only tile kernels schedule for instruction-
# level parallelism (their occupancy is bounded by LDS, not registers)
SOURCE_FLAGS = {"hydro.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]}
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument", "-Wno-unused-value"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass of hipcc does not know the device-only feature flag
    noise = "'-packed-fp32-ops' is not a recognized feature"
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if noise not in l)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{out}")
    if out.strip():
        print(out)


def build(verbose: bool = False, extra=None, jobs: int = 0, debug: bool = False) -> str:
    from concurrent.futures import ThreadPoolExecutor
    bdir = os.path.join(HERE, "_build_debug" if debug else "_build")
    lib = LIB_DEBUG if debug else LIB
    if debug:
        extra = list(extra or []) + ["-DRY_DEBUG"]
    os.makedirs(bdir, exist_ok=True)
    cmds, objs = [], []
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(bdir, s + ".o")
        cmd = [HIPCC] + flags() + SOURCE_FLAGS.get(s, []) + (extra or []) + ["-c", src, "-o", obj]
        if s.endswith(".cpp"):
            cmd = [HIPCC, "-x", "hip"] + cmd[1:]
        if verbose:
            print(" ".join(cmd), flush=True)
        cmds.append(cmd)
        objs.append(obj)
    # the sources compile independently: one compiler process each
    n = jobs or min(len(cmds), os.cpu_count() or 1, 8)
    with ThreadPoolExecutor(max_workers=max(n, 1)) as ex:
        list(ex.map(_run, cmds))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    _run(cmd)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
    print(build(verbose=True, debug=True))
