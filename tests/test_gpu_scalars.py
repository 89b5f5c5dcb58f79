"""GPU parity of the passive scalars (advected with the mass flux) against
the FP64 oracle: the same bar as the hydro variables (1e-12 relative per
cell per variable, conservation to 1e-13), the hydro variables bit-identical
to a run without scalars, and tuning invariance.
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


def compare_levels(g, o, tol=TOL):
    worst = 0.0
    for lv in g.levels:
        ng, _ = g.level_info(lv)
        assert ng == o.level_info(lv)[0]
        if ng == 0:
            continue
        Ug, Uo = g.download(lv), o.download(lv)
        assert Ug.shape == Uo.shape
        worst = max(worst, cases.rel_err(Ug, Uo))
    assert worst <= tol, worst
    return worst


def uniform_with_scalars(n, nscalar, seed=3):
    prob = W.random_smooth(n, seed=seed, mach=1.5)
    return cases.with_scalars(prob, nscalar)


@pytest.mark.parametrize("nscalar", [1, 2, 3, 4])
def test_scalars_uniform_box(ry, nscalar):
    prob = uniform_with_scalars(16, nscalar)
    g, o = ry.Hydro(prob), Oracle(prob)
    g.advance(3)
    o.advance(3)
    compare_levels(g, o)
    assert g.floors() == 0


@pytest.mark.parametrize("bc", [(W.BC_PERIODIC,) * 6, (W.BC_OUTFLOW,) * 6])
@pytest.mark.parametrize("nscalar", [2, 4])
def test_scalars_amr(ry, bc, nscalar):
    prob = cases.with_scalars(cases.amr_blob(bc=bc), nscalar)
    g, o = ry.Hydro(prob), Oracle(prob)
    g.advance(2)
    o.advance(2)
    compare_levels(g, o)


def test_scalars_leave_hydro_bit_identical(ry):
    base = cases.amr_blob()
    g0 = ry.Hydro(base)
    g2 = ry.Hydro(cases.with_scalars(base, 2))
    for g in (g0, g2):
        g.advance(3)
    for lv in g0.levels:
        np.testing.assert_array_equal(g2.download(lv)[:5], g0.download(lv))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_scalar_mass_conserved(ry, precision):
    prob = cases.with_scalars(cases.amr_blob(), 3)
    g = ry.Hydro(prob, precision)
    t0 = g.totals()
    g.advance(4)
    t1 = g.totals()
    assert len(t1) == 8
    for k in (5, 6, 7):
        assert abs(t1[k] - t0[k]) <= 1e-13 * abs(t0[k])


def test_uniform_scalar_stays_uniform(ry):
    prob = cases.with_scalars(cases.amr_blob(), 2, profiles=lambda pos: [np.full(len(pos), 0.3)] * 2)
    g = ry.Hydro(prob)
    g.advance(3)
    for lv in g.levels:
        U = g.download(lv)
        for k in (5, 6):
            np.testing.assert_allclose(U[k] / U[0], 0.3, rtol=1e-13)


def test_scalar_tunings_bit_identical_and_unsupported_rejected(ry):
    prob = cases.with_scalars(cases.amr_blob(), 2)
    ref = None
    for t in ([1, 0, 4, 1, 1], [1, 0, 4, 1, 2], [2, 0, 4, 1, 1]):
        g = ry.Hydro(prob)
        g.set_tuning(*t)
        g.advance(2)
        out = [g.download(lv) for lv in g.levels]
        if ref is None:
            ref = out
        else:
            for a, b in zip(out, ref):
                np.testing.assert_array_equal(a, b)
    g = ry.Hydro(prob)
    for bad in ([1, 1, 8, 1, 1], [1, 0, 4, 1, 4], [4, 0, 4, 1, 1]):
        with pytest.raises(ry.RyError):
            g.set_tuning(*bad)
    best, times = g.autotune()
    assert best["persistent"] == 0 and len(times) == 3


def test_mixed_scalars_within_budget(ry):
    prob = uniform_with_scalars(32, 2, seed=9)
    gf, gm = ry.Hydro(prob, "fp64"), ry.Hydro(prob, "mixed")
    gf.advance(10)
    gm.advance(10)
    Uf, Um = gf.download(prob.level_min), gm.download(prob.level_min)
    for k in (0, 5, 6):
        l1 = np.abs(Um[k] - Uf[k]).sum() / np.abs(Uf[k]).sum()
        assert l1 <= 1e-5, (k, l1)


def test_full_size_uniform128_two_scalars(ry):
    """The 128^3 benchmark box with two scalars: one coarse step against the
    oracle, every cell."""
    prob = cases.with_scalars(W.uniform(128), 2)
    g, o = ry.Hydro(prob), Oracle(prob)
    g.advance(1)
    o.advance(1)
    compare_levels(g, o)


def test_batch_rejects_scalars(ry):
    box = cases.with_scalars(W.uniform_state(8), 1)
    with pytest.raises(ry.RyError):
        ry.BatchHydro([box, box])
