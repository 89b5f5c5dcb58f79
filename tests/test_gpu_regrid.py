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


def same_mesh_and_state(a, b):
    for lv in a.levels:
        assert a.level_info(lv) == b.level_info(lv), lv
        if a.level_info(lv)[0] == 0:
            continue
        ka, ra = a.mesh(lv)
        kb, rb = b.mesh(lv)
        np.testing.assert_array_equal(ka, kb)
        np.testing.assert_array_equal(ra, rb)
        np.testing.assert_array_equal(a.download(lv), b.download(lv))


@pytest.mark.parametrize("bc", [(W.BC_PERIODIC,) * 6, (W.BC_OUTFLOW,) * 6])
def test_device_and_host_regrid_paths_bit_identical(ry, bc):
    """The all-device regrid and the host-flag path give the same mesh and
    state bit for bit, and the solver continues identically on both (the
    host builder's tile lists leave out tiles without a leaf cell, the
    device builder's keep them: neither changes a result)."""
    prob = cases.with_scalars(cases.amr_blob(bc=bc), 2)
    a, b = ry.Hydro(prob), ry.Hydro(prob)
    b.set_regrid_device(False)
    for _ in range(3):
        a.advance(1)
        b.advance(1)
        assert a.regrid() == b.regrid()
        same_mesh_and_state(a, b)
    a.advance(2)
    b.advance(2)
    same_mesh_and_state(a, b)


@pytest.mark.parametrize("bc", [(W.BC_PERIODIC,) * 6, (W.BC_OUTFLOW,) * 6])
def test_mixed_form_device_and_host_regrid_paths_bit_identical(ry, bc):
    """The mixed form through both regrid paths (all on the device, and host
    flags with the device remap): the same meshes and states bit for bit
    over three rounds of a coarse step and a regrid, and the same solution
    after two more steps."""
    prob = cases.with_scalars(cases.amr_blob(bc=bc), 1)
    a, b = ry.Hydro(prob, "mixed"), ry.Hydro(prob, "mixed")
    b.set_regrid_device(False)
    for _ in range(3):
        a.advance(1)
        b.advance(1)
        assert a.regrid() == b.regrid()
        same_mesh_and_state(a, b)
    assert a.level_info(a.levels[-1])[0] > 0
    a.advance(2)
    b.advance(2)
    same_mesh_and_state(a, b)


def test_device_regrid_empties_and_regrows_levels(ry):
    """Thresholds that remove every refined level, then restore them: counts,
    meshes and states against the oracle on the way down and back up."""
    prob = ramp_problem(5.4)
    g, o = ry.Hydro(prob), Oracle(prob)
    for thr in (1e9, 5.4, 4.6):
        g.set_refine_param(thr)
        o.set_refine_param(thr)
        assert g.regrid() == o.regrid()
        compare(g, o, 0.0)
    g.advance(1)
    o.advance(1)
    compare(g, o)


def test_zoom_full_size_device_regrid_matches_host_path(ry):
    """The zoom-in hierarchy (levels 7-12) after two coarse steps: one regrid
    on each path, bit-identical meshes and states, then one more step."""
    prob = W.zoom()
    a, b = ry.Hydro(prob), ry.Hydro(prob)
    b.set_regrid_device(False)
    a.advance(2)
    b.advance(2)
    assert a.regrid() == b.regrid()
    same_mesh_and_state(a, b)
    a.advance(1)
    b.advance(1)
    same_mesh_and_state(a, b)


@pytest.mark.parametrize("theta", [0.5, 0.3])
def test_gradient_criterion_regrid_matches_oracle(ry, theta):
    """Regrid under the gradient criterion (the two-level mesh's rule: the
    device flag kernel's neighbour-difference branch) after two coarse
    steps, and a threshold change, against the oracle: identical meshes and
    counts, states within the parity bar."""
    prob = W.twolevel(32, theta)
    g, o = ry.Hydro(prob), Oracle(prob)
    step_both(g, o, 2)
    counts = g.regrid()
    assert counts == o.regrid()
    compare(g, o)
    g.set_refine_param(0.8 * theta)
    o.set_refine_param(0.8 * theta)
    assert g.regrid() == o.regrid()
    compare(g, o)
    step_both(g, o, 1)
    compare(g, o)


@pytest.mark.parametrize("bc", [(W.BC_PERIODIC,) * 6, (W.BC_OUTFLOW,) * 6])
def test_gradient_criterion_on_refined_levels(ry, bc):
    """The gradient criterion on a refined level (levels 3-5: the device flag
    kernel reads the neighbour rule from the tile presence masks and the
    face neighbours from the tile tables): after two coarse steps and two
    threshold changes, the device regrid gives the oracle's counts and
    states, and the host-flag path's mesh and state bit for bit."""
    prob = cases.analytic_problem("gblob3-5", 3, 5, cases.blob_state, theta=0.05, bc=bc)
    g, o, h = ry.Hydro(prob), Oracle(prob), ry.Hydro(prob)
    h.set_regrid_device(False)
    for _ in range(2):   # all three with the oracle's time step
        dt = o.cfl_dt()
        for x in (o, g, h):
            x.coarse_step(dt)
    for theta in (None, 0.03, 0.08):
        if theta is not None:
            for x in (g, o, h):
                x.set_refine_param(theta)
        counts = g.regrid()
        assert counts == o.regrid() == h.regrid(), theta
        assert g.level_info(5)[0] > 0
        compare(g, o)
        same_mesh_and_state(g, h)
    step_both(g, o, 1)
    compare(g, o)


@pytest.mark.parametrize("bc", [(W.BC_PERIODIC,) * 6, (W.BC_OUTFLOW,) * 6])
def test_regrid_on_base_side_2_mod_4(ry, bc):
    """A base of 18 cells per side (9 octs per axis: blocks and tiles of the
    base cut by the domain's high side) under the gradient criterion: after
    two coarse steps and a threshold change, the device regrid gives the
    oracle's counts and states, and the host-flag path's mesh and state bit
    for bit."""
    import dataclasses
    prob = dataclasses.replace(W.twolevel(36, 0.5), bc=bc)
    g, o, h = ry.Hydro(prob), Oracle(prob), ry.Hydro(prob)
    h.set_regrid_device(False)
    for _ in range(2):   # all three with the oracle's time step
        dt = o.cfl_dt()
        for x in (o, g, h):
            x.coarse_step(dt)
    for theta in (None, 0.35):
        if theta is not None:
            for x in (g, o, h):
                x.set_refine_param(theta)
        counts = g.regrid()
        assert counts == o.regrid() == h.regrid(), theta
        assert g.level_info(prob.level_max)[0] > 0
        compare(g, o)
        same_mesh_and_state(g, h)
    step_both(g, o, 1)
    compare(g, o)


@pytest.mark.parametrize("bc", [(W.BC_PERIODIC,) * 6, (W.BC_OUTFLOW,) * 6])
def test_regrid_on_non_cubic_box(ry, bc):
    """A box of 8 x 16 x 12 base cells (levels 3-5, mass threshold): three
    rounds of a coarse step and a regrid, the device regrid giving the
    oracle's counts and states and the host-flag path's mesh and state bit
    for bit."""
    prob = cases.noncubic_blob(bc)
    g, o, h = ry.Hydro(prob), Oracle(prob), ry.Hydro(prob)
    h.set_regrid_device(False)
    for _ in range(3):
        dt = o.cfl_dt()
        for x in (o, g, h):
            x.coarse_step(dt)
        assert g.regrid() == o.regrid() == h.regrid()
        assert g.level_info(prob.level_max)[0] > 0
        compare(g, o)
        same_mesh_and_state(g, h)


@pytest.mark.parametrize("bc", [(W.BC_PERIODIC,) * 6, (W.BC_OUTFLOW,) * 6])
def test_regrid_after_upload_restricts_every_refined_cell(ry, bc):
    """A state uploaded to a refined level leaves its parents' means out of
    date; the next device regrid restricts every refined cell (after a step
    or the build only the cells above new octs need it): counts and states
    as the oracle's, mesh and state as the host-flag path's bit for bit."""
    prob = cases.amr_blob(bc=bc)
    g, o, h = ry.Hydro(prob), Oracle(prob), ry.Hydro(prob)
    h.set_regrid_device(False)
    dt = o.cfl_dt()
    for x in (o, g, h):
        x.coarse_step(dt)
    lv = prob.level_min + 1
    U = g.download(lv).copy()
    U[0] *= 1.01   # density and energy up by 1%: positive, and means change
    U[4] *= 1.01
    for x in (g, o, h):
        x.upload(lv, U)
    counts = g.regrid()
    assert counts == o.regrid() == h.regrid()
    compare(g, o)
    same_mesh_and_state(g, h)
    step_both(g, o, 1)
    compare(g, o)


def test_regrid_between_multi_step_graph_runs(ry):
    """Runs long enough for the multi-step graphs (9 = 8 + 1 steps), a regrid that reallocates
    every refined level, and another such run: the graphs captured on the
    old mesh are dropped (same result as the eager path on both meshes)."""
    prob = cases.amr_blob()
    a, b = ry.Hydro(prob), ry.Hydro(prob)
    a.set_timing(True)
    for h in (a, b):
        h.advance(9)
        h.regrid()
        h.advance(9)
    assert a.t == b.t
    for lv in a.levels:
        assert a.level_info(lv) == b.level_info(lv)
        np.testing.assert_array_equal(a.download(lv), b.download(lv))
