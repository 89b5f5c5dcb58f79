"""Pins of the oracle's regrid between coarse steps (dynamic refinement: the
paper's refine_fine step around the hydro update, Table 1).

The regrid re-applies the build's refinement criterion and neighbour rule
top-down, keeps surviving octs, fills new octs by the MinMod-linear
interpolation of their parent and drops orphaned octs.  Pinned here: the
nesting invariants, conservation, idempotence, exact reproduction of a
linear field by the interpolation, and equality of the resulting mesh with
a fresh build of the same field.
"""
import numpy as np
import pytest

import workloads as W
from oracle.ryo import Oracle

import cases


def coords_and_refined(o):
    return {lv: (o.coords(lv), o.mesh(lv)[1]) for lv in o.levels}


def check_nesting(o, periodic):
    """Every oct at l+1 sits in a refined cell of an existing oct at l; every
    refined cell has exactly one child oct, its 26 neighbour cells exist at
    its level (outside an outflow face counts as existing) and it holds the
    ordered 8-child mean of its children."""
    m = coords_and_refined(o)
    for lv in list(o.levels)[:-1]:
        xyz, ref = m[lv]
        fxyz, _ = m[lv + 1]
        nref = int(np.unpackbits(ref).sum())
        assert nref == len(fxyz)
        parent = {tuple(c): i for i, c in enumerate(xyz)}
        noct = (o.prob.nbase[0] // 2) << (lv - o.prob.level_min)
        U, Uf = o.download(lv), o.download(lv + 1)
        for k, c in enumerate(fxyz):
            po = parent[tuple(c >> 1)]
            cb = (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2)
            assert (ref[po] >> cb) & 1
            cell = np.asarray(c)                          # = the refined cell at level lv
            for d in np.ndindex(3, 3, 3):
                q = cell + np.array(d) - 1
                if periodic:
                    q = q % (2 * noct)
                elif (q < 0).any() or (q >= 2 * noct).any():
                    continue
                assert tuple(q >> 1) in parent, (lv, tuple(cell), d)
            ch = Uf[:, 8 * k:8 * k + 8]
            mean = 0.125 * (((ch[:, 0] + ch[:, 1]) + (ch[:, 2] + ch[:, 3])) + ((ch[:, 4] + ch[:, 5]) + (ch[:, 6] + ch[:, 7])))
            np.testing.assert_array_equal(U[:, 8 * po + cb], mean)


def leaf_values(o):
    """{(level, oct coords, cell): U column} over leaf cells."""
    out = {}
    for lv in o.levels:
        xyz, ref = o.coords(lv), o.mesh(lv)[1]
        U = o.download(lv)
        for k, c in enumerate(xyz):
            for cb in range(8):
                if not (ref[k] >> cb) & 1:
                    out[(lv, tuple(c), cb)] = U[:, 8 * k + cb]
    return out


@pytest.mark.parametrize("bc", [(W.BC_PERIODIC,) * 6, (W.BC_OUTFLOW,) * 6])
def test_regrid_after_steps_keeps_invariants_and_totals(bc):
    periodic = bc[0] == W.BC_PERIODIC
    o = Oracle(cases.with_scalars(cases.amr_blob(bc=bc), 1))
    o.advance(3)
    t0 = o.totals()
    before = leaf_values(o)
    created, destroyed = o.regrid()
    assert created > 0 or destroyed > 0
    check_nesting(o, periodic)
    # cells that are leaves before and after keep their values bit for bit
    after = leaf_values(o)
    common = set(before) & set(after)
    assert len(common) > 0.5 * len(after)
    for k in common:
        np.testing.assert_array_equal(after[k], before[k])
    t1 = o.totals()
    for v in range(len(t0)):
        assert abs(t1[v] - t0[v]) <= 1e-14 * max(abs(t0[v]), abs(t0).max() * 1e-3), v
    # the regridded mesh is a fixed point of the rule
    assert o.regrid() == (0, 0)
    o.advance(2)                               # and the solver runs on it
    check_nesting(o, periodic)


def ramp(pos):
    return 1.0 + 3.0 * pos[:, 0] + 2.0 * pos[:, 1] + 1.5 * pos[:, 2]


def linear_problem(rho_thr):
    """Outflow box, density linear in x, y and z, at rest, p = 1."""
    def state(pos):
        n = len(pos)
        return ramp(pos), np.zeros(n), np.zeros(n), np.zeros(n), np.ones(n)
    return cases.analytic_problem("ramp", 3, 5, state, rho_thr=rho_thr, bc=(W.BC_OUTFLOW,) * 6)


def test_new_octs_reproduce_a_linear_field_and_match_a_fresh_build():
    """Lower the threshold of a built ramp and regrid: new cells must hold
    the linear field at their centres (the MinMod interpolation is exact for
    linear data away from the clamped boundary), and the mesh must be the one
    a fresh build with the lower threshold makes (point values of the same
    field)."""
    o = Oracle(linear_problem(5.4))
    before = {lv: o.level_info(lv)[0] for lv in o.levels}
    o.set_refine_param(4.6)
    created, destroyed = o.regrid()
    assert created > 0 and destroyed == 0
    fresh = Oracle(linear_problem(4.6))
    for lv in o.levels:
        kr, rr = o.mesh(lv)
        kf, rf = fresh.mesh(lv)
        np.testing.assert_array_equal(kr, kf)
        np.testing.assert_array_equal(rr, rf)
        xyz = o.coords(lv)
        U = o.download(lv)
        n = 8 << (lv - 3)
        for ci in range(8):
            pos = np.stack([(2 * xyz[:, a] + ((ci >> a) & 1) + 0.5) / n for a in range(3)], axis=1)
            inner = ((pos > 2.0 / 8) & (pos < 6.0 / 8)).all(axis=1)   # clear of the clamped faces
            np.testing.assert_allclose(U[0, ci::8][inner], ramp(pos[inner]), rtol=1e-14)
    assert sum(o.level_info(lv)[0] for lv in o.levels) > sum(before.values())


def test_raising_the_threshold_removes_levels_and_conserves():
    o = Oracle(cases.amr_blob())
    t0 = o.totals()
    o.set_refine_param(1e9)
    created, destroyed = o.regrid()
    assert created == 0 and destroyed > 0
    assert all(o.level_info(lv)[0] == 0 for lv in list(o.levels)[1:])
    t1 = o.totals()
    np.testing.assert_allclose(t1, t0, rtol=1e-14, atol=1e-14 * np.abs(t0).max())
