"""Pins of the oracle's passive scalars (advected with the mass flux; the
paper lists metals, chemistry and dust among the fields the hydro carries,
Sec. 1 and Sec. 4).

A passive scalar s is conserved as rho*s, reconstructed like the velocity
components (MinMod slope, advective half-step predictor) and carried
through HLLC like a transverse velocity (Toro 2009, Sec. 10.6).  The pins:
HLLC special cases, the hydro variables unchanged bit for bit by carrying
scalars, a uniform scalar staying uniform, the textbook MUSCL-Hancock
closed form for 1-D advection, and conservation of scalar mass with
refluxing across coarse-fine faces.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle.ryo import Oracle, hllc, hllc_scalars

import cases


def test_hllc_scalar_special_cases():
    g = 1.4
    WL = [1.0, 0.3, -0.2, 0.1, 1.0]
    WR = [0.5, -0.1, 0.4, 0.2, 0.6]
    # scalar columns leave the hydro flux unchanged, bit for bit
    for d in range(3):
        F = hllc_scalars(WL + [0.7, 0.2], WR + [0.1, 0.2], d, g)
        np.testing.assert_array_equal(F[:5], hllc(WL, WR, d, g))
        # the same scalar on both sides: F_s = s * F_rho
        assert abs(F[6] - 0.2 * F[0]) <= 1e-15 * abs(F[0])
    # supersonic to the right: upwind flux rho_L u_L s_L
    WLs, WRs = [1.0, 5.0, 0.0, 0.0, 1.0, 0.25], [0.8, 4.0, 0.0, 0.0, 0.9, 0.75]
    F = hllc_scalars(WLs, WRs, 0, g)
    assert F[5] == 1.0 * 5.0 * 0.25
    # stationary contact: no scalar flux at all
    F = hllc_scalars([1.0, 0.0, 0.0, 0.0, 1.0, 0.9], [0.1, 0.0, 0.0, 0.0, 1.0, 0.1], 0, g)
    assert F[5] == 0.0 and F[0] == 0.0


def test_scalars_leave_hydro_bit_exact():
    base = cases.amr_blob()
    o0 = Oracle(base)
    o2 = Oracle(cases.with_scalars(base, 2))
    for o in (o0, o2):
        o.advance(2)
    for lv in o0.levels:
        np.testing.assert_array_equal(o2.download(lv)[:5], o0.download(lv))


def test_uniform_scalar_stays_uniform():
    prob = cases.with_scalars(cases.amr_blob(), 3,
                              profiles=lambda pos: [np.full(len(pos), 0.3)] * 3)
    o = Oracle(prob)
    o.advance(2)
    for lv in o.levels:
        U = o.download(lv)
        for k in (5, 6, 7):
            np.testing.assert_allclose(U[k] / U[0], 0.3, rtol=1e-13)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_scalar_linear_advection_closed_form(axis):
    """Uniform rho, p and velocity u along `axis`: each column along the
    axis follows the textbook MUSCL-Hancock update for linear advection,
    s_{L,i+1/2} = s_i + (1 - lambda u) D_i / 2 with MinMod slopes D."""
    n, u, p, g = 32, 0.7, 1.0, 1.4
    x = (np.arange(n) + 0.5) / n
    s1 = 0.5 + 0.3 * np.sin(2 * np.pi * x) + 0.2 * (x > 0.6)
    shape = [2, 2, 2]
    shape[2 - axis] = n                           # array axes are (z, y, x)
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    rho = np.ones(shape)
    vel = [0 * rho, 0 * rho, 0 * rho]
    vel[axis] = np.full_like(rho, u)
    U = W.conserved(rho, vel[0], vel[1], vel[2], np.full_like(rho, p), g)
    U = np.concatenate([U, np.broadcast_to(s1.reshape(bshape), shape)[None]], axis=0)
    nb = [2, 2, 2]
    nb[axis] = n
    prob = W.Problem("advect_s", 5, 5, tuple(nb), g, U, nscalar=1)
    o = Oracle(prob)
    dt = 0.3 / n
    o.coarse_step(dt)
    Uo = o.download(5)
    xyz = o.coords(5)
    got = np.zeros(n)
    for ci in range(8):
        got[2 * xyz[:, axis] + ((ci >> axis) & 1)] = Uo[5, ci::8]
    lam = dt * nb[0]                              # dx = boxlen / nbase[0]
    a = s1 - np.roll(s1, 1)
    b = np.roll(s1, -1) - s1
    d = np.where((a > 0) & (b > 0), np.minimum(a, b), np.where((a < 0) & (b < 0), np.maximum(a, b), 0.0))
    face = s1 + 0.5 * (1 - lam * u) * d          # s_{L,i+1/2}
    expect = s1 - lam * u * (face - np.roll(face, 1))
    np.testing.assert_allclose(got, expect, rtol=1e-13, atol=0)


@pytest.mark.parametrize("bc", [(W.BC_PERIODIC,) * 6])
def test_scalar_mass_conserved_across_levels(bc):
    prob = cases.with_scalars(cases.amr_blob(bc=bc), 2)
    o = Oracle(prob)
    t0 = o.totals()
    o.advance(3)
    t1 = o.totals()
    assert len(t1) == 7
    for k in (5, 6):
        assert abs(t1[k] - t0[k]) <= 1e-13 * abs(t0[k])
