"""Full-size GPU checks of every workload in both precision forms.

FP64 form: against the oracle at the parity bar (1e-12 relative per cell,
meshes bit-exact).  Mixed FP32-bulk / FP64-update form: its relative L1
density error over the leaf cells stays within 1e-5 after the workload's
steps, measured against the FP64 oracle (or, for the zoom hierarchy's ten
coarse steps, against the GPU's FP64 form, itself pinned to the oracle for
one coarse step here); its maximum relative density and pressure errors and
its total-energy drift are checked against looser sanity bounds.
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from oracle.ryo import Oracle

import cases

pytestmark = pytest.mark.gpu

TOL = 1e-12
L1_BUDGET = 1e-5          # mixed form: relative L1 density error after the run
MAX_BOUND = 1e-3          # mixed form: sanity bound on the largest relative rho / p error


@pytest.fixture(scope="module")
def ry():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_14631_amd import ry as mod
    mod.lib()
    return mod


def compare_levels(g, o, tol=TOL):
    worst = 0.0
    for lv in g.levels:
        ng, leaf_g = g.level_info(lv)
        no, leaf_o = o.level_info(lv)
        assert (ng, leaf_g) == (no, leaf_o), lv
        if ng == 0:
            continue
        kg, rg = g.mesh(lv)
        ko, ro = o.mesh(lv)
        np.testing.assert_array_equal(kg, ko)
        np.testing.assert_array_equal(rg, ro)
        worst = max(worst, cases.rel_err(g.download(lv), o.download(lv)))
    assert worst <= tol, worst
    return worst


def check_mixed(stats, drift=None):
    print(stats, drift, flush=True)
    assert stats["l1_rho_rel"] <= L1_BUDGET, stats
    assert stats["max_rho_rel"] <= MAX_BOUND and stats["max_p_rel"] <= MAX_BOUND, stats
    if drift is not None:
        assert drift <= 1e-12, drift


def energy_drift(e0, e1):
    return abs(e1 - e0) / abs(e0)


# ------------------------------------------------------------ uniform 128^3
def test_mixed_uniform128_ten_steps_vs_oracle(ry):
    prob = W.uniform(128)
    m, o = ry.Hydro(prob, "mixed"), Oracle(prob)
    e0 = m.totals()[4]
    m.advance(prob.n_steps)
    o.advance(prob.n_steps)
    assert abs(m.t - o.t) <= 1e-6 * o.t
    check_mixed(cases.form_errors(cases.level_states(m), cases.level_states(o), prob.gamma),
                energy_drift(e0, m.totals()[4]))
    assert m.floors() == 0


# ------------------------------------------------------------- two-level AMR
def test_twolevel128_theta01_full_size_config_steps(ry):
    """The literal threshold theta = 0.1 (99% of the base refined) over its
    10 coarse steps: meshes bit-exact, FP64 within the parity bar."""
    prob = W.twolevel(128, 0.1)
    g, o = ry.Hydro(prob), Oracle(prob)
    assert g.level_info(7)[0] == o.level_info(7)[0] > 250_000
    g.advance(1)
    o.advance(1)
    compare_levels(g, o)
    g.advance(prob.n_steps - 1)
    o.advance(prob.n_steps - 1)
    assert abs(g.t - o.t) <= 1e-13 * o.t
    compare_levels(g, o)
    assert g.floors() == 0


@pytest.mark.parametrize("theta", [0.70, 0.1])
def test_mixed_twolevel128_ten_coarse_steps_vs_oracle(ry, theta):
    prob = W.twolevel(128, theta)
    m, o = ry.Hydro(prob, "mixed"), Oracle(prob)
    e0 = m.totals()[4]
    m.advance(prob.n_steps)
    o.advance(prob.n_steps)
    assert abs(m.t - o.t) <= 1e-6 * o.t
    check_mixed(cases.form_errors(cases.level_states(m), cases.level_states(o), prob.gamma),
                energy_drift(e0, m.totals()[4]))


# ------------------------------------------------------------------ zoom AMR
def test_zoom_full_size_step_regrid_step(ry):
    """Zoom-in hierarchy (levels 7-12, about 2M octs): one coarse step in
    FP64 (parity bar) and in the mixed form (budget), one device regrid
    against the oracle's (counts and meshes bit-exact, state within the
    parity bar), one more coarse step on the new mesh."""
    prob = W.zoom()
    g, m, o = ry.Hydro(prob), ry.Hydro(prob, "mixed"), Oracle(prob)
    assert g.level_info(12)[0] > 0
    g.advance(1)
    m.advance(1)
    o.advance(1)
    compare_levels(g, o)
    assert g.floors() == 0
    check_mixed(cases.form_errors(cases.level_states(m), cases.level_states(o), prob.gamma))
    m.close()
    counts = g.regrid()
    assert counts == o.regrid() and counts[0] > 10_000 and counts[1] > 10_000, counts
    compare_levels(g, o)
    g.advance(1)
    o.advance(1)
    compare_levels(g, o)


def test_mixed_zoom_ten_coarse_steps_vs_fp64(ry):
    prob = W.zoom()
    f, m = ry.Hydro(prob), ry.Hydro(prob, "mixed")
    e0f, e0m = f.totals()[4], m.totals()[4]
    f.advance(prob.n_steps)
    m.advance(prob.n_steps)
    assert abs(m.t - f.t) <= 1e-6 * f.t
    stats = cases.form_errors(cases.level_states(m), cases.level_states(f), prob.gamma)
    check_mixed(stats, energy_drift(e0m, m.totals()[4]))
    assert energy_drift(e0f, f.totals()[4]) <= 1e-12


# ----------------------------------------------------------- batched boxes
def test_mixed_batch512_sampled_boxes_vs_oracle(ry):
    """All 512 uneven boxes, 20 steps in the mixed form; 16 boxes spread
    over the list recomputed by the oracle in FP64."""
    boxes = W.batch(512)
    bh = ry.BatchHydro(boxes, "mixed")
    bh.run(20)
    worst = 0.0
    for b in range(0, 512, 32):
        o = Oracle(boxes[b])
        o.advance(20)
        ref = [(o.download(1), np.zeros(o.level_info(1)[0], np.uint8), 1.0)]
        got = [(bh.download(b), ref[0][1], 1.0)]
        s = cases.form_errors(got, ref, boxes[b].gamma)
        check_mixed(s)
        worst = max(worst, s["l1_rho_rel"])
        assert abs(bh.box_info(b)[1] - o.t) <= 1e-6 * o.t
    print("worst sampled-box L1 density error", worst)
