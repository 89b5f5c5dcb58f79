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
VALU_PEAK_ISSUE = 1024 * 2.4e9 / 4      # 256 CUs x 4 SIMDs, one wave64 instruction per 4 cycles
BYTES_PER_CELL_UPDATE = 80
METRIC = "hydro cell-updates/s (FP64 vs mixed FP32) + % HBM roofline, 128^3 and zoom AMR"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("hydro_tile.h", "hydro.hip", "ry_internal.h"):
        with open(os.path.join(ROOT, "paper_2411_14631_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
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


def time_advance(h, steps, warmup, timing):
    import torch
    h.set_timing(timing)
    if warmup:
        h.advance(warmup)
    if timing:
        h.set_timing(False)
        h.set_timing(True)          # reset the per-kernel accumulators
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.advance(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = h.kernel_time("hydro") if timing else (0, 0.0)
    h.set_timing(False)
    return dt, kt


def cell_updates_per_coarse_step(h):
    tot = 0
    for k, lv in enumerate(h.levels):
        _, leaf = h.level_info(lv)
        tot += leaf << k
    return tot


def run_uniform(precision, steps, warmup, tune, fixed=None, eager_only=False):
    import workloads as W
    from paper_2411_14631_amd import Hydro
    prob = W.uniform(128)
    h = Hydro(prob, precision)
    tuning = None
    if fixed:
        h.set_tuning(*fixed)
    elif tune:
        tuning, _ = h.autotune()
    cups = cell_updates_per_coarse_step(h)
    e0 = h.totals()[4]
    if eager_only:
        # every launch of the run with HIP events around it (profiling runs:
        # the profiler's per-kernel average then covers the same launches)
        dt_graph, pcie = None, None
        dt_ev, (nl, ms) = time_advance(h, steps, warmup, timing=True)
    else:
        dt_graph, _ = time_advance(h, steps, warmup, timing=False)
        dt_ev, (nl, ms) = time_advance(h, steps, 0, timing=True)
        pcie = pcie_inclusive(h, steps)
    return dict(prob=prob, h=h, cups=cups, dt_graph=dt_graph, dt_timed=dt_ev, launches=nl, kernel_ms=ms,
                tuning=tuning or h.tuning(), floors=h.floors(), e0=e0, pcie=pcie)


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


def run_zoom(prob, precision, steps, tune):
    from paper_2411_14631_amd import Hydro
    t0 = time.perf_counter()
    h = Hydro(prob, precision)
    build_s = time.perf_counter() - t0
    if tune:
        h.autotune()
    cups = cell_updates_per_coarse_step(h)
    noct = sum(h.level_info(lv)[0] for lv in h.levels)
    e0 = h.totals()[4]
    # two untimed steps capture the single-step graphs of both state
    # parities, so that the timed steps replay graphs (fewer than 8 timed
    # steps: no multi-step graph is captured inside the timed region)
    assert steps < 8
    dt_graph, _ = time_advance(h, steps, 2, timing=False)
    h.advance(10 - steps - 2)                      # 10 coarse steps in total
    return dict(h=h, cups=cups, noct=noct, dt=dt_graph, build_s=build_s, e0=e0, floors=h.floors(),
                levels={lv: h.level_info(lv) for lv in h.levels})


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
        dt, _ = time_advance(h, steps, warmup, timing=False)
        _, (nl, ms) = time_advance(h, steps, 0, timing=True)
        k = ms / max(nl, 1)
        gbs = 16 * (5 + nscalar) * cups / (k * 1e-3) / 1e9
        res[prec] = {"value": cups * steps / dt, "unit": "cell-updates/s", "kernel_avg_ms": round(k, 5),
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-zoom", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-poisson", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--tuning", type=str, default="",
                    help="fixed hydro tuning tiles_per_wg,persistent,waves_per_cu,batch,waves_per_tile")
    ap.add_argument("--only", choices=["fp64", "mixed", "poisson"], default=None)
    ap.add_argument("--eager-only", action="store_true",
                    help="with --only fp64/mixed: every step launched eagerly with HIP events (for profiling)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="first launch a plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on exactly one GPU (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design only", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    tune = not args.no_tune
    fixed = [int(x) for x in args.tuning.split(",")] if args.tuning else None

    if args.copy_probe_mb:
        import workloads as W
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
    if args.only:
        log(f"bench: uniform 128^3 {args.only} only")
        r = run_uniform(args.only, args.steps, args.warmup, tune, fixed, args.eager_only)
        ms = r["kernel_ms"] / max(r["launches"], 1)
        print(json.dumps({"precision": args.only,
                          "cell_updates_per_s": r["cups"] * args.steps / (r["dt_graph"] or r["dt_timed"]),
                          "timed_cell_updates_per_s": r["cups"] * args.steps / r["dt_timed"],
                          "hydro_kernel_avg_ms": ms, "tuning": r["tuning"]}), flush=True)
        return

    log("bench: uniform 128^3 fp64")
    f = run_uniform("fp64", args.steps, args.warmup, tune, fixed)
    log("bench: uniform 128^3 mixed")
    m = run_uniform("mixed", args.steps, args.warmup, tune, fixed)

    # value: the production path (one coarse step per captured graph, no
    # per-kernel events); the kernel average comes from the second timed run
    # of the same steps with HIP events around every launch
    value = f["cups"] * args.steps / f["dt_graph"]
    ms_per_step = 1e3 * f["dt_graph"] / args.steps
    kernel_avg_ms = f["kernel_ms"] / max(f["launches"], 1)
    alg_bytes = BYTES_PER_CELL_UPDATE * f["cups"]          # one launch per coarse step
    achieved = alg_bytes / (kernel_avg_ms * 1e-3) / 1e9
    traffic = traffic_from_profiles("uniform128_fp64")
    # VALU issue: wave64 instructions per launch (profiled counter) over the
    # live kernel time, against 1,024 SIMDs x 2.4 GHz / 4 cycles per wave64
    # instruction
    valu_insts = profiled_counters("uniform128_fp64").get("valu_insts_per_launch")
    valu = None
    if valu_insts:
        rate = valu_insts / (kernel_avg_ms * 1e-3)
        valu = {"unit": "wave64 VALU instructions/s", "instructions_per_launch": valu_insts,
                "achieved": round(rate, -6), "peak": VALU_PEAK_ISSUE, "frac": round(rate / VALU_PEAK_ISSUE, 4)}
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "hydro_kernel<double>", "kernel_avg_ms": round(kernel_avg_ms, 5),
                "alg_bytes_per_launch": alg_bytes}

    m_kernel_ms = m["kernel_ms"] / max(m["launches"], 1)
    mixed = {"value": m["cups"] * args.steps / m["dt_graph"], "unit": "cell-updates/s",
             "kernel_avg_ms": round(m_kernel_ms, 5),
             "hbm_frac": round(BYTES_PER_CELL_UPDATE * m["cups"] / (m_kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
             "timed_value": m["cups"] * args.steps / m["dt_timed"], "tuning": m["tuning"]}
    # mixed vs fp64 after the same number of steps (both ran warmup + 2 x steps)
    mixed["vs_fp64"] = compare_forms(f["h"], m["h"], f["e0"], m["e0"])
    mixed["steps_compared"] = args.warmup + 2 * args.steps
    del f["h"], m["h"]
    torch.cuda.empty_cache()

    zoom = None
    if not args.no_zoom:
        import workloads as W
        zprob = W.zoom()
        zoom = {}
        handles = {}
        for prec in ("fp64", "mixed"):
            log(f"bench: zoom AMR {prec}")
            z = run_zoom(zprob, prec, 3, tune)
            zoom[prec] = {"value": z["cups"] * 3 / z["dt"], "unit": "cell-updates/s",
                          "hbm_frac": round(BYTES_PER_CELL_UPDATE * z["cups"] * 3 / z["dt"] / 1e9 / HBM_PEAK_GBS, 4),
                          "cell_updates_per_coarse_step": z["cups"], "octs": z["noct"],
                          "ms_per_coarse_step": round(1e3 * z["dt"] / 3, 3), "build_s": round(z["build_s"], 1),
                          "floor_activations": z["floors"]}
            zoom["levels"] = {str(k): v for k, v in z["levels"].items()}
            handles[prec] = z
        zoom["mixed_vs_fp64_after_10_coarse_steps"] = compare_forms(
            handles["fp64"]["h"], handles["mixed"]["h"], handles["fp64"]["e0"], handles["mixed"]["e0"])
        # one regrid of each evolved mesh (FP64: all on the device; mixed: the
        # host-flag path, for comparison), then one coarse step on it
        for prec, on_device in (("fp64", True), ("mixed", False)):
            h = handles[prec]["h"]
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
        del handles, z, h
        torch.cuda.empty_cache()

    # two-level AMR: 64^3 base under the 128^3 field, gradient criterion at
    # the primary threshold (about a quarter refined) and at the literal 0.1
    twolevel = None
    if not args.no_zoom:
        import workloads as W
        twolevel = {}
        for theta in (0.70, 0.1):
            tprob = W.twolevel(128, theta)
            entry = {}
            for prec in ("fp64", "mixed"):
                log(f"bench: two-level AMR theta {theta} {prec}")
                z = run_zoom(tprob, prec, 7, tune)
                entry[prec] = {"value": z["cups"] * 7 / z["dt"], "unit": "cell-updates/s",
                               "hbm_frac": round(BYTES_PER_CELL_UPDATE * z["cups"] * 7 / z["dt"] / 1e9 / HBM_PEAK_GBS,
                                                 4),
                               "cell_updates_per_coarse_step": z["cups"], "octs": z["noct"],
                               "ms_per_coarse_step": round(1e3 * z["dt"] / 7, 3), "floor_activations": z["floors"]}
                entry["levels"] = {str(k): v for k, v in z["levels"].items()}
                del z
            twolevel[f"theta_{theta}"] = entry
        torch.cuda.empty_cache()

    batch = None
    if not args.no_zoom:
        import workloads as W
        from paper_2411_14631_amd import BatchHydro
        boxes = W.batch(512)
        cells = sum(p.nbase[0] ** 3 for p in boxes)
        batch = {"boxes": 512, "cells": cells, "steps": 20}
        for prec in ("fp64", "mixed"):
            log(f"bench: batch 512 boxes {prec}")
            bh = BatchHydro(boxes, prec)
            btune = bh.autotune()[0] if tune else bh.tuning()
            bh.run(20)                                  # warm-up: captures the 20-step graph
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bh.run(20)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            batch[prec] = {"value": cells * 20 / el, "unit": "cell-updates/s", "ms_per_step": 1e3 * el / 20,
                           "hbm_frac": round(BYTES_PER_CELL_UPDATE * cells * 20 / el / 1e9 / HBM_PEAK_GBS, 4),
                           "tuning": btune}
            bh.close()
            del bh
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
                   "timed_value": f["cups"] * args.steps / f["dt_timed"], "floor_activations": f["floors"],
                   "pcie_inclusive_value": f["pcie"]},
        "roofline": roofline,
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
