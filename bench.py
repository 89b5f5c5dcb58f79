"""Benchmark of the octree hydro step on one MI355X.

Prints ONE JSON line.  Headline: FP64 hydro cell-updates/s on the uniform
128^3 periodic lognormal box (262144 octs, gamma 5/3, CFL 0.8); a step is
one coarse step of the whole hot path (device CFL/dt, the fused per-tile
MUSCL-Hancock/HLLC update with its CFL epilogue).  Also reported: the mixed
FP32/FP64 form on the same box, the zoom-shaped AMR workload (levels 7-12,
both forms), the roofline of the dominant (hydro) kernel from HIP events on
its launch stream, and the CPU oracle timed on the host as a baseline.

A cell-update is one leaf cell advanced by one step of its own level;
algorithmic HBM bytes are 80 per cell-update (5 FP64 read + 5 written).

Timing: every throughput figure is the median of REPS repetitions of its
timed steps (each repetition bracketed by device synchronisations), taken
after the warm-up steps and an untimed settling period of the workload's own
steps (--settle-ms, 200 ms by default: the GPU's clocks need tens of
milliseconds of load to reach their sustained level); a plain
device copy timed in the same run gives the achievable HBM bandwidth next to
the vendor peak.  Every mixed-form figure carries its errors against the
FP64 form after the workload's own step count (10 coarse steps; 20 for the
batched boxes): relative L1 and largest relative density and pressure
errors over leaf cells, and both forms' total-energy drift.  The FP64 form
is itself pinned to the oracle by the GPU tests, and the CPU-baseline leg
compares both forms with the oracle directly on the 128^3 box.

The line also carries the uniform-level Poisson solver (PPCG with the
seven-point preconditioner) on a 256^3 periodic gravity source: iterations
to eps = 1e-4 against pipelined plain CG, time to solution, and the
iteration kernel's rate against HBM (128 algorithmic bytes per cell and
iteration: the eight recurrence vectors read and written once).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
REPS = 5                                # timed repetitions per figure (median reported)
COPY_PROBE_BYTES = 256 << 20
VALU_PEAK_ISSUE = 1024 * 2.4e9 / 4      # 256 CUs x 4 SIMDs, one wave64 instruction per 4 cycles
BYTES_PER_CELL_UPDATE = 80
METRIC = "hydro cell-updates/s (FP64 vs mixed FP32) + % HBM roofline, 128^3 and zoom AMR"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the hydro kernel's sources with comments and blank space
    removed (a comment edit leaves the profiled counters valid; any change
    of code does not)."""
    import re
    h = hashlib.sha256()
    for f in ("hydro_tile.h", "hydro.hip", "ry_internal.h"):
        with open(os.path.join(ROOT, "paper_2411_14631_amd", "csrc", f), encoding="utf-8") as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def profiled_counters(workload_key):
    """rocprofv3 counter figures per hydro launch (HBM bytes, VALU
    instructions), if they were taken on the current kernel source (else {})."""
    path = os.path.join(ROOT, "profiles", "hydro_traffic.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        d = json.load(f)
    e = d.get(workload_key)
    if not e or e.get("kernel_hash") != kernel_source_hash():
        return {}
    return e


def traffic_from_profiles(workload_key):
    """HBM bytes per hydro launch measured with rocprofv3 counters (or None)."""
    return profiled_counters(workload_key).get("bytes_per_launch")


def median(v):
    v = sorted(v)
    n = len(v)
    return v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])


# Untimed settling before each timed section: the workload's own steps, back
# to back, for at least this many milliseconds, so that the GPU's clocks have
# reached their sustained level (on the 128^3 box the step time falls from
# 0.119 to 0.098 ms over the first ~25 ms of back-to-back steps, then stays).
SETTLE_MS = 200.0


def set_settle_ms(ms):
    global SETTLE_MS
    SETTLE_MS = float(ms)


def settle(step, ms=None):
    """Run `step()` (a few of the workload's steps) until `ms` milliseconds
    of wall time have passed; returns the number of calls."""
    import torch
    ms = SETTLE_MS if ms is None else ms
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n = 0
    while (time.perf_counter() - t0) * 1e3 < ms:
        step()
        torch.cuda.synchronize()
        n += 1
    return n


def timed_reps(h, steps, reps=REPS):
    """Wall time of `steps` coarse steps (graph replay, the production path),
    `reps` times; returns (median seconds, all repetitions)."""
    import torch
    h.set_timing(False)
    out = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.advance(steps)
        torch.cuda.synchronize()
        out.append(time.perf_counter() - t0)
    return median(out), out


def eager_kernel_time(h, steps, name="hydro"):
    """`steps` coarse steps launched one kernel at a time with HIP events on
    the library's stream around every launch: (launches, total ms) of the
    kernels called `name`."""
    import torch
    h.set_timing(False)
    h.set_timing(True)
    torch.cuda.synchronize()
    h.advance(steps)
    torch.cuda.synchronize()
    kt = h.kernel_time(name)
    h.set_timing(False)
    return kt


def cell_updates_per_coarse_step(h):
    tot = 0
    for k, lv in enumerate(h.levels):
        _, leaf = h.level_info(lv)
        tot += leaf << k
    return tot


def level_tunings(h):
    return {str(lv): h.level_tuning(lv) for lv in h.levels}


def tuning_label(t):
    if t["tile_cells"] == 8:
        return f"8^3-cell tile (4x4x4 octs), {64 * t['waves_per_tile']} threads"
    return (f"4^3-cell tile (2x2x2 octs), {64 * t['waves_per_tile']} threads per tile, "
            f"{t['tiles_per_wg']} tile(s) per workgroup" + (", queue-fed" if t["persistent"] else ""))


def make(prob, precision, tune, fixed):
    from paper_2411_14631_amd import Hydro
    t0 = time.perf_counter()
    h = Hydro(prob, precision)
    build_s = time.perf_counter() - t0
    if fixed:
        h.set_tuning(*fixed)
    elif tune:
        h.autotune()
    return h, build_s


def pcie_inclusive(h, steps):
    """Cell-updates/s when the state crosses PCIe both ways: upload the
    current state from the host, advance `steps` coarse steps, download."""
    import torch
    lv = h.prob.level_min
    U = h.download(lv)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.upload(lv, U)
    h.advance(steps)
    h.download(lv)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return cell_updates_per_coarse_step(h) * steps / el


def run_amr_pair(prob, tune, fixed, timed_steps, eager_steps=0, keep=False):
    """Both precision forms of one (AMR or uniform) workload: each advanced
    its configuration's coarse steps (the first ones capture the graphs),
    compared, then timed (median of REPS repetitions of `timed_steps`)."""
    import torch
    res, hs = {}, {}
    for prec in ("fp64", "mixed"):
        h, build_s = make(prob, prec, tune, fixed)
        e0 = h.totals()[4]
        h.advance(prob.n_steps)
        hs[prec] = (h, e0)
        # floor activations over the configuration's coarse steps (the later
        # settling and timed steps add their own)
        res[prec] = {"build_s": round(build_s, 2), "tunings": level_tunings(h),
                     "floor_activations": h.floors(), "floor_activations_steps": prob.n_steps}
    res["mixed"]["vs_fp64"] = compare_forms(hs["fp64"][0], hs["mixed"][0], hs["fp64"][1], hs["mixed"][1])
    res["mixed"]["vs_fp64"]["coarse_steps"] = prob.n_steps
    for prec in ("fp64", "mixed"):
        h = hs[prec][0]
        cups = cell_updates_per_coarse_step(h)
        settle(lambda: h.advance(8))
        med, reps = timed_reps(h, timed_steps)
        r = res[prec]
        r.update({"value": cups * timed_steps / med, "unit": "cell-updates/s",
                  "ms_per_coarse_step": round(1e3 * med / timed_steps, 4),
                  "hbm_frac": round(BYTES_PER_CELL_UPDATE * cups * timed_steps / med / 1e9 / HBM_PEAK_GBS, 4),
                  "cell_updates_per_coarse_step": cups, "timed_coarse_steps": timed_steps,
                  "repetitions_ms_per_coarse_step": [round(1e3 * x / timed_steps, 4) for x in reps],
                  "octs": sum(h.level_info(lv)[0] for lv in h.levels)})
        if eager_steps:
            # the hydro kernels' own time per coarse step (HIP events around
            # each launch): their rate against HBM without launch gaps
            nl, ms = eager_kernel_time(h, eager_steps)
            hk = ms / eager_steps
            r["hydro_kernels_ms_per_coarse_step"] = round(hk, 4)
            r["hydro_kernels_hbm_frac"] = round(BYTES_PER_CELL_UPDATE * cups / (hk * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
            r["hydro_launches_per_coarse_step"] = nl // eager_steps
    res["levels"] = {str(lv): hs["fp64"][0].level_info(lv) for lv in hs["fp64"][0].levels}
    if keep:
        return res, hs
    for prec in hs:
        hs[prec][0].close()
    del hs
    torch.cuda.empty_cache()
    return res, None


def run_zoom_only(precision, steps, warmup, tune, fixed, eager):
    """The zoom hierarchy alone (for profiling): `warmup` untimed coarse
    steps, then `steps` timed ones, replayed from captured graphs or, with
    `eager`, launched one by one with HIP events around every kernel (the
    hydro kernels' summed time per coarse step then gives the hydro
    kernels' rate against HBM)."""
    import torch
    import workloads as W
    h, _ = make(W.zoom(), precision, tune, fixed)
    cups = cell_updates_per_coarse_step(h)
    if warmup:
        h.advance(warmup)
    settle(lambda: h.advance(1))
    out = {"workload": "zoom AMR levels 7-12", "precision": precision, "steps": steps,
           "cell_updates_per_coarse_step": cups, "tunings": level_tunings(h),
           "levels": {str(lv): h.level_info(lv) for lv in h.levels}}
    if eager:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nl, ms = eager_kernel_time(h, steps)
        dt = time.perf_counter() - t0
        hydro_ms = ms / steps
        out.update({"hydro_launches": nl, "hydro_ms_per_coarse_step": hydro_ms,
                    "hydro_achieved_GBps": BYTES_PER_CELL_UPDATE * cups / (hydro_ms * 1e-3) / 1e9})
        out["hydro_hbm_frac"] = out["hydro_achieved_GBps"] / HBM_PEAK_GBS
    else:
        dt, _ = timed_reps(h, steps, 1)
    out.update({"value": cups * steps / dt, "ms_per_coarse_step": 1e3 * dt / steps})
    h.close()
    return out


def run_regrid_only(steps, warmup, tune, fixed):
    """The zoom hierarchy's device regrid alone (for profiling): `warmup`
    coarse steps, then `steps` rounds of one coarse step and one timed
    regrid."""
    import torch
    import workloads as W
    h, _ = make(W.zoom(), "fp64", tune, fixed)
    h.set_regrid_device(True)
    h.advance(max(1, warmup))
    times, counts = [], []
    for _ in range(steps):
        h.advance(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        created, destroyed = h.regrid()
        times.append(time.perf_counter() - t0)
        counts.append((created, destroyed))
        log(f"bench: regrid {1e3 * times[-1]:.2f} ms, created {created}, destroyed {destroyed}")
    out = {"workload": "zoom AMR levels 7-12, device regrid", "steps": steps,
           "octs": sum(h.level_info(lv)[0] for lv in h.levels),
           "regrid_ms": [round(1e3 * t, 3) for t in times], "created_destroyed": counts}
    h.close()
    return out


def leaf_fields(h):
    """Leaf-cell density, pressure and cell volume of every level."""
    import numpy as np
    g = h.prob.gamma
    out = []
    for k, lv in enumerate(h.levels):
        n, _ = h.level_info(lv)
        if n == 0:
            continue
        U = h.download(lv)
        _, ref = h.mesh(lv)
        leaf = ~np.unpackbits(ref[:, None], axis=1, bitorder="little").astype(bool).reshape(-1)
        rho = U[0][leaf]
        p = (g - 1.0) * (U[4][leaf] - 0.5 * (U[1][leaf] ** 2 + U[2][leaf] ** 2 + U[3][leaf] ** 2) / rho)
        vol = (h.prob.boxlen / (h.prob.nbase[0] << k)) ** 3
        out.append((rho, p, vol))
    return out


def compare_forms(hf, hm, e0f, e0m):
    """Mixed form against the FP64 form (which is pinned to the oracle):
    relative L1 and max errors of density and pressure over leaf cells, and
    each form's total-energy drift."""
    import numpy as np
    a, b = leaf_fields(hf), leaf_fields(hm)
    l1 = sum(np.abs(rm - rf).sum() * v for (rf, _, v), (rm, _, _) in zip(a, b))
    norm = sum(np.abs(rf).sum() * v for (rf, _, v) in a)
    mx_r = max(float(np.max(np.abs(rm - rf) / np.abs(rf))) for (rf, _, _), (rm, _, _) in zip(a, b))
    mx_p = max(float(np.max(np.abs(pm - pf) / np.abs(pf))) for (_, pf, _), (_, pm, _) in zip(a, b))
    l1p = sum(np.abs(pm - pf).sum() * v for (_, pf, v), (_, pm, _) in zip(a, b)) / \
        sum(np.abs(pf).sum() * v for (_, pf, v) in a)
    ef, em = hf.totals()[4], hm.totals()[4]
    return {"l1_rho_rel": float(l1 / norm), "max_rho_rel": mx_r, "l1_p_rel": float(l1p), "max_p_rel": mx_p,
            "energy_drift_fp64": float(abs(ef - e0f) / abs(e0f)), "energy_drift_mixed": float(abs(em - e0m) / abs(e0m))}


def compare_batches(bf, bm, boxes):
    """Mixed-form boxes against the FP64 boxes after the same steps: relative
    L1 (cell-volume weighted, each box a unit box) and largest relative
    errors of density and pressure over every box's cells, and each form's
    total-energy drift summed over the boxes."""
    import numpy as np
    l1r = l1p = nr = npr = e0 = ef = em = 0.0
    mr = mp = 0.0
    for b, p in enumerate(boxes):
        g = p.gamma
        vol = 1.0 / p.nbase[0] ** 3
        Uf, Um = bf.download(b), bm.download(b)

        def rho_p(U):
            return U[0], (g - 1.0) * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0])
        rf, pf = rho_p(Uf)
        rm, pm = rho_p(Um)
        l1r += np.abs(rm - rf).sum() * vol
        l1p += np.abs(pm - pf).sum() * vol
        nr += np.abs(rf).sum() * vol
        npr += np.abs(pf).sum() * vol
        mr = max(mr, float(np.max(np.abs(rm - rf) / np.abs(rf))))
        mp = max(mp, float(np.max(np.abs(pm - pf) / np.abs(pf))))
        e0 += p.U_base[4].sum() * vol
        ef += Uf[4].sum() * vol
        em += Um[4].sum() * vol
    return {"l1_rho_rel": float(l1r / nr), "max_rho_rel": mr, "l1_p_rel": float(l1p / npr), "max_p_rel": mp,
            "energy_drift_fp64": float(abs(ef - e0) / abs(e0)), "energy_drift_mixed": float(abs(em - e0) / abs(e0)),
            "steps": 20}


def cpu_baseline(budget_s=12.0):
    """The oracle, as it is, on the host: 128^3 uniform box, whole steps
    until about budget_s of wall time."""
    import workloads as W
    from oracle.ryo import Oracle, lib
    prob = W.uniform(128)
    o = Oracle(prob)
    cores = lib().ryo_num_threads()
    e0 = o.totals()[4]
    n = 0
    t0 = time.perf_counter()
    while True:
        o.advance(1)
        n += 1
        el = time.perf_counter() - t0
        if el > budget_s or n >= 100:
            break
    cups = 128 ** 3 * n / el
    # the oracle's state after these n steps: the reference for the GPU
    # forms' accuracy on the same workload (reported below, untimed)
    ref = {"U": o.download(prob.level_min), "t": o.t, "drift": abs(o.totals()[4] - e0) / abs(e0), "n": n}
    # the same oracle on one thread, a few steps
    lib().ryo_set_num_threads(1)
    n1 = 0
    t0 = time.perf_counter()
    while True:
        o.advance(1)
        n1 += 1
        el1 = time.perf_counter() - t0
        if el1 > budget_s / 2 or n1 >= 20:
            break
    lib().ryo_set_num_threads(cores)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": cups, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"uniform 128^3 periodic box, {n} whole coarse steps ({el:.1f} s wall)"
                      + (f" on {model}" if model else ""),
            "value_one_thread": 128 ** 3 * n1 / el1,
            "gpu_vs_oracle": gpu_vs_oracle(prob, ref)}


def gpu_vs_oracle(prob, ref):
    """Both GPU forms advanced as many steps as the oracle took: relative
    L1 and max errors of density and pressure against the oracle's state,
    the time reached, and each code's total-energy drift."""
    import numpy as np
    import torch
    from paper_2411_14631_amd import Hydro
    g = prob.gamma

    def rho_p(U):
        return U[0], (g - 1.0) * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0])

    rr, pr = rho_p(ref["U"])
    out = {"steps": ref["n"], "oracle_energy_drift": float(ref["drift"])}
    for prec in ("fp64", "mixed"):
        h = Hydro(prob, prec)
        e0 = h.totals()[4]
        h.advance(ref["n"])
        rg, pg = rho_p(h.download(prob.level_min))
        out[prec] = {"l1_rho_rel": float(np.abs(rg - rr).sum() / np.abs(rr).sum()),
                     "max_rho_rel": float(np.max(np.abs(rg - rr) / np.abs(rr))),
                     "l1_p_rel": float(np.abs(pg - pr).sum() / np.abs(pr).sum()),
                     "max_p_rel": float(np.max(np.abs(pg - pr) / np.abs(pr))),
                     "t_rel": float(abs(h.t - ref["t"]) / ref["t"]),
                     "energy_drift": float(abs(h.totals()[4] - e0) / abs(e0))}
        h.close()
        del h
        torch.cuda.empty_cache()
    return out


def run_scalars(nscalar=2, steps=10, warmup=2):
    """Uniform 128^3 box carrying passive scalars: both precision forms, HIP
    events on the hydro kernel; algorithmic bytes 16 per variable and
    cell-update (5 + nscalar variables read and written)."""
    import torch
    import workloads as W
    from paper_2411_14631_amd import Hydro
    prob = W.uniform(128, nscalar=nscalar)
    res = {"workload": f"uniform 128^3 periodic lognormal box with {nscalar} passive scalars",
           "nscalar": nscalar, "alg_bytes_per_cell_update": 16 * (5 + nscalar)}
    for prec in ("fp64", "mixed"):
        h = Hydro(prob, prec)
        tuning, _ = h.autotune()
        cups = cell_updates_per_coarse_step(h)
        h.advance(warmup)
        settle(lambda: h.advance(8))
        med, _ = timed_reps(h, steps)
        nl, ms = eager_kernel_time(h, steps)
        k = ms / max(nl, 1)
        gbs = 16 * (5 + nscalar) * cups / (k * 1e-3) / 1e9
        res[prec] = {"value": cups * steps / med, "unit": "cell-updates/s", "kernel_avg_ms": round(k, 5),
                     "achieved_GBps": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "tuning": tuning}
        h.close()
        del h
        torch.cuda.empty_cache()
    return res


POISSON_BYTES_PER_CELL = 128


def run_poisson(n=256, eps=1e-4, timed_iters=20):
    """PPCG vs pipelined plain CG on the n^3 periodic gravity source."""
    import torch
    import workloads as W
    from paper_2411_14631_amd import ry
    b = W.poisson_source(n)
    N = n ** 3
    res = {"workload": f"{n}^3 periodic lognormal gravity source, FP64, eps target {eps:g}", "cells": N,
           "alg_bytes_per_iteration": POISSON_BYTES_PER_CELL * N}
    for name, pc in (("ppcg", ry.RY_PC_STENCIL7), ("cg", ry.RY_PC_NONE)):
        g = ry.Poisson(b.shape, ry.RY_PBC_PERIODIC, pc)
        g.set_rhs(b)
        g.solve(eps, 5000)                      # warm-up (graph capture, clocks)
        g.set_rhs(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = g.solve(eps, 5000)
        torch.cuda.synchronize()
        solve_s = time.perf_counter() - t0
        eps_reached = float(g.eps_history()[-1])
        g.set_rhs(b)
        g.set_timing(True)
        g.iterate(timed_iters)
        nl, ms = g.kernel_time()
        g.set_timing(False)
        kern_ms = ms / max(nl, 1)
        achieved = POISSON_BYTES_PER_CELL * N / (kern_ms * 1e-3) / 1e9
        res[name] = {"iterations": k, "eps_reached": eps_reached, "solve_ms": round(1e3 * solve_s, 3),
                     "ms_per_iteration": round(1e3 * solve_s / max(k, 1), 4),
                     "kernel_avg_ms": round(kern_ms, 5), "achieved_GBps": round(achieved, 1),
                     "hbm_frac": round(achieved / HBM_PEAK_GBS, 4)}
        g.close()
        del g
        torch.cuda.empty_cache()
    res["iteration_ratio_cg_over_ppcg"] = round(res["cg"]["iterations"] / max(res["ppcg"]["iterations"], 1), 3)
    res["paper_iteration_ratio"] = 1.86
    res["roofline"] = {"bound": "hbm", "kernel": "ppcg_iterate_kernel<stencil7>",
                       "achieved": res["ppcg"]["achieved_GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": res["ppcg"]["hbm_frac"]}
    return res


def copy_probe():
    """A plain device copy of COPY_PROBE_BYTES (read + write), timed in this
    run: the achievable HBM bandwidth next to the vendor peak."""
    import workloads as W
    from paper_2411_14631_amd import Hydro
    probe = Hydro(W.uniform_state(8), "fp64")
    settle(lambda: probe.copy_probe(COPY_PROBE_BYTES, reps=20))
    ms = probe.copy_probe(COPY_PROBE_BYTES, reps=20)
    probe.close()
    gbs = 2 * COPY_PROBE_BYTES / (ms * 1e-3) / 1e9
    return {"bytes_copied": COPY_PROBE_BYTES, "ms": round(ms, 5), "GBps": round(gbs, 1),
            "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4), "kernel": "ry::copy_kernel (16-byte loads and stores)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--settle-ms", type=float, default=SETTLE_MS,
                    help="untimed back-to-back steps before each timed section, in ms of wall time "
                         "(GPU clocks reach their sustained level)")
    ap.add_argument("--no-zoom", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-poisson", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tuning", type=str, default="",
                    help="fixed hydro tuning tiles_per_wg,persistent,waves_per_cu,batch,waves_per_tile[,tile_cells]")
    ap.add_argument("--only", choices=["fp64", "mixed", "poisson", "zoom", "zoom-mixed", "batch", "batch-mixed",
                                       "twolevel", "twolevel-mixed", "regrid"], default=None)
    ap.add_argument("--eager-only", action="store_true",
                    help="with --only: every step launched eagerly with HIP events (for profiling)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first launch a plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    set_settle_ms(args.settle_ms)
    if args.gpus != 1:
        print(f"bench.py: the library runs on exactly one GPU (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design only", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    import workloads as W
    tune = not args.no_tune
    fixed = [int(x) for x in args.tuning.split(",")] if args.tuning else None

    if args.copy_probe_mb:
        from paper_2411_14631_amd import Hydro
        probe = Hydro(W.uniform_state(8), "fp64")
        ms = probe.copy_probe(args.copy_probe_mb << 20, reps=5)
        log(f"bench: copy probe {args.copy_probe_mb} MiB: {ms:.4f} ms "
            f"({2 * (args.copy_probe_mb << 20) / (ms * 1e-3) / 1e9:.1f} GB/s)")
        probe.close()

    if args.only == "poisson":
        log("bench: poisson 256^3 only")
        print(json.dumps(run_poisson()), flush=True)
        return
    if args.only in ("batch", "batch-mixed"):
        # the 512 batched boxes alone (profiling): `warmup` untimed 20-step
        # runs (graph capture), then one timed 20-step run
        from paper_2411_14631_amd import BatchHydro
        prec = "mixed" if args.only == "batch-mixed" else "fp64"
        boxes = W.batch(512)
        cells = sum(p.nbase[0] ** 3 for p in boxes)
        bh = BatchHydro(boxes, prec)
        if fixed:
            bh.set_tuning(*fixed)
        elif tune:
            bh.autotune()
        for _ in range(max(args.warmup, 1)):
            bh.run(20)
        settle(lambda: bh.run(20))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bh.run(20)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(json.dumps({"workload": "512 batched boxes", "precision": prec, "tuning": bh.tuning(),
                          "value": cells * 20 / el, "ms_per_step": 1e3 * el / 20}), flush=True)
        return
    if args.only in ("twolevel", "twolevel-mixed"):
        prec = "mixed" if args.only == "twolevel-mixed" else "fp64"
        log(f"bench: two-level theta 0.70 {prec} only")
        h, _ = make(W.twolevel(128, 0.70), prec, tune, fixed)
        cups = cell_updates_per_coarse_step(h)
        h.advance(max(args.warmup, 2))
        settle(lambda: h.advance(8))
        med, _ = timed_reps(h, args.steps)
        print(json.dumps({"workload": "two-level theta 0.70", "precision": prec, "tunings": level_tunings(h),
                          "value": cups * args.steps / med, "ms_per_coarse_step": 1e3 * med / args.steps}), flush=True)
        h.close()
        return
    if args.only == "regrid":
        log("bench: zoom device regrid only")
        print(json.dumps(run_regrid_only(args.steps, args.warmup, tune, fixed)), flush=True)
        return
    if args.only in ("zoom", "zoom-mixed"):
        prec = "mixed" if args.only == "zoom-mixed" else "fp64"
        log(f"bench: zoom AMR {prec} only")
        print(json.dumps(run_zoom_only(prec, args.steps, args.warmup, tune, fixed, args.eager_only)), flush=True)
        return
    if args.only:
        log(f"bench: uniform 128^3 {args.only} only")
        h, _ = make(W.uniform(128), args.only, tune, fixed)
        cups = cell_updates_per_coarse_step(h)
        h.advance(args.warmup)
        settle(lambda: h.advance(8))
        out = {"precision": args.only, "tuning": h.tuning()}
        if args.eager_only:
            # every launch of the run with HIP events around it (profiling runs:
            # the profiler's per-kernel average then covers the same launches)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nl, ms = eager_kernel_time(h, args.steps)
            out["timed_cell_updates_per_s"] = cups * args.steps / (time.perf_counter() - t0)
            out["hydro_kernel_avg_ms"] = ms / max(nl, 1)
        else:
            med, _ = timed_reps(h, args.steps)
            out["cell_updates_per_s"] = cups * args.steps / med
        print(json.dumps(out), flush=True)
        return

    log("bench: copy probe")
    probe = copy_probe()

    # ---- headline: uniform 128^3, FP64 and mixed
    uprob = W.uniform(128)
    hs = {}
    for prec in ("fp64", "mixed"):
        log(f"bench: uniform 128^3 {prec}")
        h, build_s = make(uprob, prec, tune, fixed)
        e0 = h.totals()[4]
        h.advance(uprob.n_steps)                 # the configuration's 10 steps (captures the graphs)
        hs[prec] = (h, e0, h.floors())
    mixed_err = compare_forms(hs["fp64"][0], hs["mixed"][0], hs["fp64"][1], hs["mixed"][1])
    mixed_err["steps"] = uprob.n_steps
    res = {}
    for prec in ("fp64", "mixed"):
        h = hs[prec][0]
        cups = cell_updates_per_coarse_step(h)
        h.advance(args.warmup)
        settle(lambda: h.advance(8))
        med, reps = timed_reps(h, args.steps)                 # value: graph replay, the production path
        nl, ms = eager_kernel_time(h, args.steps)             # the kernel's own time (HIP events)
        res[prec] = dict(cups=cups, med=med, reps=reps, kernel_ms=ms / max(nl, 1), tuning=h.tuning(),
                         floors=hs[prec][2], pcie=pcie_inclusive(h, args.steps) if prec == "fp64" else None)
    for prec in hs:
        hs[prec][0].close()
    del hs, h
    torch.cuda.empty_cache()

    f, m = res["fp64"], res["mixed"]
    value = f["cups"] * args.steps / f["med"]
    ms_per_step = 1e3 * f["med"] / args.steps
    alg_bytes = BYTES_PER_CELL_UPDATE * f["cups"]          # one launch per coarse step
    achieved = alg_bytes / (f["kernel_ms"] * 1e-3) / 1e9
    pkey = f"uniform128_fp64_k{f['tuning']['tile_cells']}"
    traffic = traffic_from_profiles(pkey)
    # VALU issue: wave64 instructions per launch (profiled counter) over the
    # live kernel time, against 1,024 SIMDs x 2.4 GHz / 4 cycles per wave64
    # instruction
    valu_insts = profiled_counters(pkey).get("valu_insts_per_launch")
    valu = None
    if valu_insts:
        rate = valu_insts / (f["kernel_ms"] * 1e-3)
        valu = {"unit": "wave64 VALU instructions/s", "instructions_per_launch": valu_insts,
                "achieved": round(rate, -6), "peak": VALU_PEAK_ISSUE, "frac": round(rate / VALU_PEAK_ISSUE, 4)}
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "hydro_kernel<double> (" + tuning_label(f["tuning"]) + ")",
                "kernel_avg_ms": round(f["kernel_ms"], 5), "alg_bytes_per_launch": alg_bytes,
                "achievable_GBps": probe["GBps"], "frac_of_achievable": round(achieved / probe["GBps"], 4)}
    mixed = {"value": m["cups"] * args.steps / m["med"], "unit": "cell-updates/s",
             "kernel_avg_ms": round(m["kernel_ms"], 5),
             "hbm_frac": round(BYTES_PER_CELL_UPDATE * m["cups"] / (m["kernel_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "tuning": m["tuning"], "repetitions_ms_per_step": [round(1e3 * x / args.steps, 4) for x in m["reps"]],
             "vs_fp64": mixed_err}

    zoom = None
    if not args.no_zoom:
        log("bench: zoom AMR fp64 + mixed")
        zoom, zh = run_amr_pair(W.zoom(), tune, fixed, timed_steps=8, eager_steps=2, keep=True)
        # one regrid of each evolved mesh (FP64: all on the device; mixed: the
        # host-flag path, for comparison), then one coarse step on it
        for prec, on_device in (("fp64", True), ("mixed", False)):
            h = zh[prec][0]
            h.set_regrid_device(on_device)
            before = sum(h.level_info(lv)[0] for lv in h.levels)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            created, destroyed = h.regrid()
            rg = time.perf_counter() - t0
            after = sum(h.level_info(lv)[0] for lv in h.levels)
            h.advance(1)
            zoom[f"regrid_{prec}"] = {
                "ms": round(1e3 * rg, 2), "octs_before": before, "octs_after": after, "created": created,
                "destroyed": destroyed,
                "path": "device" if on_device else "host flags and tables, device state remap"}
        for prec in zh:
            zh[prec][0].close()
        del zh
        torch.cuda.empty_cache()

    # two-level AMR: 64^3 base under the 128^3 field, gradient criterion at
    # the primary threshold (about a quarter refined) and at the literal 0.1
    twolevel = None
    if not args.no_zoom:
        twolevel = {}
        for theta in (0.70, 0.1):
            log(f"bench: two-level AMR theta {theta}")
            twolevel[f"theta_{theta}"], _ = run_amr_pair(W.twolevel(128, theta), tune, fixed, timed_steps=8,
                                                         eager_steps=2)

    batch = None
    if not args.no_zoom:
        from paper_2411_14631_amd import BatchHydro
        boxes = W.batch(512)
        cells = sum(p.nbase[0] ** 3 for p in boxes)
        batch = {"boxes": 512, "cells": cells, "steps": 20}
        bhs = {}
        for prec in ("fp64", "mixed"):
            log(f"bench: batch 512 boxes {prec}")
            bh = BatchHydro(boxes, prec)
            btune = bh.autotune()[0] if tune else bh.tuning()
            bh.run(20)                                  # the workload's 20 steps (captures the graph)
            bhs[prec] = bh
            batch[prec] = {"tuning": btune}
        batch["mixed"]["vs_fp64"] = compare_batches(bhs["fp64"], bhs["mixed"], boxes)
        for prec in ("fp64", "mixed"):
            bh = bhs[prec]
            settle(lambda: bh.run(20))
            el = []
            for _ in range(REPS):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                bh.run(20)
                torch.cuda.synchronize()
                el.append(time.perf_counter() - t0)
            med = median(el)
            batch[prec].update({"value": cells * 20 / med, "unit": "cell-updates/s", "ms_per_step": 1e3 * med / 20,
                                "hbm_frac": round(BYTES_PER_CELL_UPDATE * cells * 20 / med / 1e9 / HBM_PEAK_GBS, 4),
                                "repetitions_ms_per_step": [round(1e3 * x / 20, 4) for x in el]})
            bh.close()
        del bhs, bh
        torch.cuda.empty_cache()

    scalars = None
    if not args.no_zoom:
        log("bench: uniform 128^3 with 2 passive scalars")
        scalars = run_scalars()

    poisson = None
    if not args.no_poisson:
        log("bench: poisson 256^3 ppcg vs cg")
        poisson = run_poisson()

    cpu = None
    if not args.no_cpu:
        log("bench: cpu oracle baseline")
        cpu = cpu_baseline()

    out = {
        "metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "uniform 128^3 periodic lognormal box (262144 octs), FP64, gamma 5/3, CFL 0.8",
                   "cells": 128 ** 3, "cell_updates_per_step": f["cups"], "tuning": f["tuning"],
                   "repetitions": REPS, "settle_ms_before_timing": SETTLE_MS, "repetitions_ms_per_step": [round(1e3 * x / args.steps, 4) for x in f["reps"]],
                   "floor_activations": f["floors"], "floor_activations_steps": uprob.n_steps,
                   "pcie_inclusive_value": f["pcie"]},
        "roofline": roofline,
        "copy_probe": probe,
        "valu_issue": valu,
        "cpu_baseline": cpu,
        "mixed": mixed,
        "zoom_amr": zoom,
        "twolevel_amr": twolevel,
        "batch_boxes": batch,
        "passive_scalars": scalars,
        "poisson": poisson,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
