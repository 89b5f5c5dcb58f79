"""GPU parity of the regrid between coarse steps (ry_regrid) against the
oracle's (ryo_regrid): bit-exact meshes (Hilbert keys, refined-cell masks)
and created / destroyed counts, state within 1e-12 relative, conservation,
idempotence, and the solver continuing on the regridded mesh.
"""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W
from oracle.ryo import Oracle

import cases

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def ry():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_14631_amd import ry as mod
    mod.lib()
    return mod


def compare(g, o, tol=TOL):
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


def step_both(g, o, n):
    for _ in range(n):
        dt = o.cfl_dt()
        assert abs(g.cfl_dt() - dt) <= 1e-14 * dt
        o.coarse_step(dt)
        g.coarse_step(dt)


@pytest.mark.parametrize("bc", [(W.BC_PERIODIC,) * 6, (W.BC_OUTFLOW,) * 6])
def test_regrid_after_steps_matches_oracle(ry, bc):
    prob = cases.with_scalars(cases.amr_blob(bc=bc), 1)
    g, o = ry.Hydro(prob), Oracle(prob)
    step_both(g, o, 3)
    t0 = g.totals()
    counts = g.regrid()
    assert counts == o.regrid()
    assert counts[0] > 0 or counts[1] > 0
    compare(g, o)
    t1 = g.totals()
    for v in range(len(t0)):
        assert abs(t1[v] - t0[v]) <= 1e-14 * max(abs(t0[v]), 1e-3 * np.abs(t0).max())
    assert g.regrid() == (0, 0) == o.regrid()
    step_both(g, o, 2)                        # the solver runs on the new mesh
    compare(g, o)


def test_regrid_every_coarse_step_graph_path(ry):
    """advance / regrid alternation through the captured-graph path, both
    precision forms run; FP64 against the oracle."""
    prob = cases.amr_blob()
    g, o = ry.Hydro(prob), Oracle(prob)
    m = ry.Hydro(prob, "mixed")
    for _ in range(3):
        g.advance(1)
        o.advance(1)
        m.advance(1)
        assert g.regrid() == o.regrid()
        m.regrid()
    compare(g, o)
    for lv in g.levels:
        assert m.level_info(lv)[0] > 0 or g.level_info(lv)[0] == 0


def ramp_problem(rho_thr):
    def state(pos):
        n = len(pos)
        return (1.0 + 3.0 * pos[:, 0] + 2.0 * pos[:, 1] + 1.5 * pos[:, 2], np.zeros(n), np.zeros(n),
                np.zeros(n), np.ones(n))
    return cases.analytic_problem("ramp", 3, 5, state, rho_thr=rho_thr, bc=(W.BC_OUTFLOW,) * 6)


@pytest.mark.parametrize("new_thr", [4.6, 9.0, 1e9])
def test_threshold_change_matches_oracle(ry, new_thr):
    prob = ramp_problem(5.4)
    g, o = ry.Hydro(prob), Oracle(prob)
    g.set_refine_param(new_thr)
    o.set_refine_param(new_thr)
    assert g.regrid() == o.regrid()
    compare(g, o, 0.0)                        # same arithmetic in the same order: bit-exact
    g.advance(1)
    o.advance(1)
    compare(g, o)


def test_regrid_inside_a_coarse_step_is_refused(ry):
    prob = cases.amr_blob()
    g = ry.Hydro(prob)
    dt = g.cfl_dt()
    g.hydro_step(prob.level_max, 0.25 * dt)
    with pytest.raises(ry.RyError):
        g.regrid()
