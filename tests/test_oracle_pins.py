"""Pins of the FP64 CPU oracle against facts that do not come from itself:
published values, closed forms, invariants, an exact Riemann solver and an
independent dense brute-force AMR stepper.  CPU only."""
from __future__ import annotations

import math
import os
import warnings

import numpy as np
import pytest

import workloads as W
from oracle.ryo import Oracle, hilbert_key, hllc, minmod

import cases
import exact_riemann as ER
from bruteforce_amr import DenseAMR

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    rows = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.split("#")[0].split()
            if line:
                rows[line[0]] = [float(x) for x in line[1:]]
    return rows


# ----------------------------------------------------------------- Hilbert
def test_hilbert_order1_matches_gray_code():
    rows = read_golden("hilbert_order1.txt")
    for k, (x, y, z) in rows.items():
        assert hilbert_key(1, int(x), int(y), int(z)) == int(k)


@pytest.mark.parametrize("bits", [1, 2, 3, 4])
def test_hilbert_bijective_and_face_adjacent(bits):
    n = 1 << bits
    pts = {}
    for z in range(n):
        for y in range(n):
            for x in range(n):
                pts[hilbert_key(bits, x, y, z)] = (x, y, z)
    assert sorted(pts) == list(range(n ** 3))
    for h in range(n ** 3 - 1):
        a, b = np.array(pts[h]), np.array(pts[h + 1])
        assert np.abs(a - b).sum() == 1, (h, a, b)
    assert pts[0] == (0, 0, 0)


def test_hilbert_subcubes_are_contiguous():
    bits = 4
    n = 1 << bits
    for s in (2, 4, 8):
        for z0 in range(0, n, s):
            for y0 in range(0, n, s):
                for x0 in range(0, n, s):
                    keys = sorted(hilbert_key(bits, x, y, z) for x in range(x0, x0 + s)
                                  for y in range(y0, y0 + s) for z in range(z0, z0 + s))
                    assert keys[-1] - keys[0] == s ** 3 - 1
                    assert keys[0] % (s ** 3) == 0


# ------------------------------------------------------------ limiter, HLLC
def test_minmod_cases():
    assert minmod(1.0, 2.0) == 1.0
    assert minmod(2.0, 1.0) == 1.0
    assert minmod(-1.0, -3.0) == -1.0
    assert minmod(-3.0, -1.0) == -1.0
    assert minmod(1.0, -1.0) == 0.0
    assert minmod(0.0, 5.0) == 0.0
    assert minmod(-2.0, 0.0) == 0.0
    assert minmod(1e-300, 1e-300) == 1e-300   # no product underflow


def physical_flux(Wv, d, g):
    r, p = Wv[0], Wv[4]
    u = Wv[1 + d]
    E = p / (g - 1) + 0.5 * r * (Wv[1] ** 2 + Wv[2] ** 2 + Wv[3] ** 2)
    F = np.zeros(5)
    F[0] = r * u
    F[1:4] = r * u * np.array(Wv[1:4])
    F[1 + d] += p
    F[4] = (E + p) * u
    return F


@pytest.mark.parametrize("d", [0, 1, 2])
def test_hllc_consistency_equal_states(d):
    rng = np.random.default_rng(11 + d)
    for _ in range(50):
        Wv = [rng.uniform(0.1, 3), *rng.uniform(-3, 3, 3), rng.uniform(0.1, 3)]
        F = hllc(Wv, Wv, d, 1.4)
        np.testing.assert_allclose(F, physical_flux(Wv, d, 1.4), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_hllc_stationary_contact_exact(d):
    WL = [2.0, 0.0, 0.0, 0.0, 0.7]
    WR = [0.3, 0.0, 0.0, 0.0, 0.7]
    WL[1 + (d + 1) % 3] = 0.4   # tangential velocity jumps too
    F = hllc(WL, WR, d, 5 / 3)
    assert F[0] == 0.0 and F[4] == 0.0
    assert F[1 + d] == 0.7


def test_hllc_moving_contact_is_upwind():
    # isolated contact (equal u, p): HLLC resolves it exactly -> upwind flux
    WL = [1.5, 0.4, 0.1, -0.2, 1.0]
    WR = [0.2, 0.4, -0.3, 0.5, 1.0]
    np.testing.assert_allclose(hllc(WL, WR, 0, 1.4), physical_flux(WL, 0, 1.4), rtol=1e-13)
    WL[1], WR[1] = -0.4, -0.4
    np.testing.assert_allclose(hllc(WL, WR, 0, 1.4), physical_flux(WR, 0, 1.4), rtol=1e-13)


def test_hllc_supersonic_upwind():
    WL = [1.0, 5.0, 0.0, 0.0, 1.0]
    WR = [0.5, 4.0, 0.0, 0.0, 0.8]
    np.testing.assert_array_equal(hllc(WL, WR, 0, 1.4), physical_flux(WL, 0, 1.4))
    WL = [1.0, -5.0, 0.0, 0.0, 1.0]
    WR = [0.5, -6.0, 0.0, 0.0, 0.8]
    np.testing.assert_array_equal(hllc(WL, WR, 0, 1.4), physical_flux(WR, 0, 1.4))


def test_hllc_matches_alternative_star_form():
    """Toro's alternative star-flux form (see bruteforce_amr) agrees with the
    oracle's F_K + S_K (U*_K - U_K) form on random states."""
    dense = DenseAMR(2, 1, 1.4, 0.8, (0,) * 6)
    rng = np.random.default_rng(5)
    for d in range(3):
        WL = np.stack([rng.uniform(0.1, 3, 200), *rng.uniform(-2, 2, (3, 200)), rng.uniform(0.1, 3, 200)])
        WR = np.stack([rng.uniform(0.1, 3, 200), *rng.uniform(-2, 2, (3, 200)), rng.uniform(0.1, 3, 200)])
        Fd = dense.hllc(WL, WR, d)
        for i in range(200):
            Fo = hllc(WL[:, i], WR[:, i], d, 1.4)
            scale = np.abs(Fo).max()
            np.testing.assert_allclose(Fo, Fd[:, i], rtol=0, atol=1e-13 * scale)


def test_hllc_mirror_symmetry():
    rng = np.random.default_rng(3)
    for _ in range(100):
        WL = np.array([rng.uniform(0.1, 3), *rng.uniform(-2, 2, 3), rng.uniform(0.1, 3)])
        WR = np.array([rng.uniform(0.1, 3), *rng.uniform(-2, 2, 3), rng.uniform(0.1, 3)])
        F = hllc(WL, WR, 0, 1.4)
        mL, mR = WR.copy(), WL.copy()
        mL[1] *= -1
        mR[1] *= -1
        Fm = hllc(mL, mR, 0, 1.4)
        expect = -F
        expect[1] = F[1]
        np.testing.assert_allclose(Fm, expect, rtol=0, atol=1e-14 * np.abs(F).max())


# ---------------------------------------------------------------- Sod (P1)
def test_golden_sod_star_state():
    rows = read_golden("sod_star_toro.txt")
    ps, us = ER.star_state(1.0, 0.0, 1.0, 0.125, 0.0, 0.1, 1.4)
    rl, rr = ER.star_densities(1.0, 1.0, 0.125, 0.1, ps, 1.4)
    for name, val in (("p_star", ps), ("u_star", us), ("rho_star_L", rl), ("rho_star_R", rr)):
        ref, tol = rows[name]
        assert abs(val - ref) <= tol, (name, val, ref)


def sod_tube(n):
    p = W.sod(32)
    x = (np.arange(n) + 0.5) / n
    left = np.broadcast_to((x < 0.5)[None, None, :], (2, 2, n))
    rho = np.where(left, 1.0, 0.125)
    pr = np.where(left, 1.0, 0.1)
    z = np.zeros_like(rho)
    U = W.conserved(rho, z, z, z, pr, 1.4)
    lvl = int(round(math.log2(n)))
    return W.Problem(f"sodtube{n}", lvl, lvl, (n, 2, 2), 1.4, U, bc=p.bc, t_end=0.1)


def test_sod_3d_columns_bit_identical_and_exact():
    prob = W.sod(32)
    o = Oracle(prob)
    nsteps = o.advance(1000, prob.t_end)
    assert o.t == 0.1 and 14 <= nsteps <= 20
    assert o.floors() == 0
    U = o.download(5)
    xyz = o.coords(5)
    dense = np.zeros((5, 32, 32, 32))
    for ci in range(8):
        X = 2 * xyz[:, 0] + (ci & 1)
        Y = 2 * xyz[:, 1] + ((ci >> 1) & 1)
        Z = 2 * xyz[:, 2] + ((ci >> 2) & 1)
        dense[:, X, Y, Z] = U[:, ci::8]
    col = dense[:, :, 0, 0]
    for y in range(32):
        for z in range(32):
            np.testing.assert_array_equal(dense[:, :, y, z], col)
    np.testing.assert_array_equal(dense[2], 0.0)
    np.testing.assert_array_equal(dense[3], 0.0)
    exact = ER.cell_average_density(1, 0, 1, 0.125, 0, 0.1, 1.4, 0.5, 0.1, 32)
    l1 = np.abs(col[0] - exact).mean()
    assert l1 < 0.02, l1


def test_sod_convergence_and_wave_positions():
    errs = []
    for n in (32, 64, 128, 256):
        o = Oracle(sod_tube(n))
        o.advance(100000, 0.1)
        U = o.download(o.prob.level_min)
        xyz = o.coords(o.prob.level_min)
        rho = np.zeros(n)
        for ci in range(8):
            rho[2 * xyz[:, 0] + (ci & 1)] = U[0, ci::8]
        exact = ER.cell_average_density(1, 0, 1, 0.125, 0, 0.1, 1.4, 0.5, 0.1, n)
        errs.append(np.abs(rho - exact).mean())
        if n == 256:
            # shock: last cell with rho > 0.2 of the right plateau within 2 cells of 0.6752
            x = (np.arange(n) + 0.5) / n
            shock = x[np.where(rho > 0.5 * (0.26557 + 0.125))[0].max()]
            assert abs(shock - 0.6752) < 2.0 / n
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[-1] < 0.004, errs


# --------------------------------------------------------- invariants (P2-5)
def dense_level(o, level):
    U = o.download(level)
    xyz = o.coords(level)
    n = o.prob.nbase[0] << (level - o.prob.level_min)
    out = np.full((5, n, n, n), np.nan)
    for ci in range(8):
        out[:, 2 * xyz[:, 0] + (ci & 1), 2 * xyz[:, 1] + ((ci >> 1) & 1), 2 * xyz[:, 2] + ((ci >> 2) & 1)] = U[:, ci::8]
    return out


def test_uniform_state_preserved_bit_exact():
    prob = W.uniform_state(8)
    o = Oracle(prob)
    U0 = o.download(3)
    o.advance(5)
    np.testing.assert_array_equal(o.download(3), U0)


def test_uniform_state_preserved_on_amr_bit_exact():
    prob = cases.analytic_problem(
        "amr_uniform", 3, 5,
        lambda pos: (np.full(len(pos), 1.3), np.full(len(pos), 0.3), np.full(len(pos), -0.2),
                     np.full(len(pos), 0.1), np.full(len(pos), 0.7)),
        rho_thr=1.0)
    # threshold below rho refines where the neighbour rule allows: force a
    # partial refinement by using a position-dependent threshold via GRAD=0
    o = Oracle(prob)
    n4, _ = o.level_info(4)
    assert n4 > 0
    before = [o.download(l) for l in o.levels]
    o.advance(3)
    for l, U0 in zip(o.levels, before):
        np.testing.assert_array_equal(o.download(l), U0)


def test_stationary_contact_preserved_bit_exact():
    n = 16
    g = W.smooth_gaussian_field(n, 99, 1.5)
    rho = np.exp(0.8 * g)
    z = np.zeros_like(rho)
    U = W.conserved(rho, z, z, z, np.full_like(rho, 0.6), 1.4)
    prob = W.Problem("contact", 4, 4, (n, n, n), 1.4, U)
    o = Oracle(prob)
    U0 = o.download(4)
    o.advance(4)
    np.testing.assert_array_equal(o.download(4), U0)


def test_stationary_contact_preserved_on_amr_bit_exact():
    def state(pos):
        d = pos - 0.5
        rho = 1.0 + 30.0 * np.exp(-(d * d).sum(1) / 0.01) + 0.5 * np.sin(6.28 * pos[:, 1])
        z = np.zeros(len(pos))
        return rho, z, z, z, np.full(len(pos), 2.0)
    prob = cases.analytic_problem("contact_amr", 3, 5, state, rho_thr=2.0)
    o = Oracle(prob)
    assert o.level_info(5)[0] > 0
    before = [o.download(l) for l in o.levels]
    o.advance(3)
    for l, U0 in zip(o.levels, before):
        np.testing.assert_array_equal(o.download(l), U0)


def check_conservation(o, steps):
    t0 = o.totals()
    msum = 0.0
    for l in o.levels:
        U = o.download(l)
        msum += np.abs(U[1:4]).sum() * (1.0 / (o.prob.nbase[0] << (l - o.prob.level_min))) ** 3
    o.advance(steps)
    t1 = o.totals()
    assert abs(t1[0] - t0[0]) <= 1e-13 * abs(t0[0])
    assert abs(t1[4] - t0[4]) <= 1e-13 * abs(t0[4])
    for v in (1, 2, 3):
        assert abs(t1[v] - t0[v]) <= 1e-13 * msum


def test_conservation_periodic_uniform():
    o = Oracle(W.random_smooth(16))
    check_conservation(o, 5)
    assert o.floors() == 0


def test_conservation_periodic_amr():
    o = Oracle(cases.amr_blob())
    assert o.level_info(5)[0] > 0
    check_conservation(o, 3)


def permuted_problem(prob, perm, flip_x=False):
    """Relabel axes (perm = new order of old axes) and optionally mirror x."""
    U = prob.U_base.copy()                   # (5, z, y, x)
    # to (5, x, y, z)
    A = np.transpose(U, (0, 3, 2, 1))
    mom = A[1:4].copy()
    A = np.concatenate([A[:1], mom[list(perm)], A[4:]])
    A = np.transpose(A, (0,) + tuple(1 + p for p in perm))
    if flip_x:
        A = A[:, ::-1].copy()
        A[1] = -A[1]
    Ub = np.ascontiguousarray(np.transpose(A, (0, 3, 2, 1)))
    return W.Problem(prob.name + "_perm", prob.level_min, prob.level_max, prob.nbase, prob.gamma, Ub,
                     bc=prob.bc)


def test_mirror_and_permutation_symmetry():
    prob = W.random_smooth(16, seed=21, mach=1.5)
    o = Oracle(prob)
    o.advance(3)
    ref = dense_level(o, 4)
    om = Oracle(permuted_problem(prob, (0, 1, 2), flip_x=True))
    om.advance(3)
    m = dense_level(om, 4)[:, ::-1]
    m[1] = -m[1]
    assert cases.rel_err(m.reshape(5, -1), ref.reshape(5, -1)) < 1e-13
    op = Oracle(permuted_problem(prob, (1, 2, 0)))
    op.advance(3)
    pm = dense_level(op, 4)              # axes (x', y', z') = old (y, z, x)
    back = np.transpose(pm, (0, 3, 1, 2))  # -> old (x, y, z)
    mom = back[1:4]
    back = np.concatenate([back[:1], mom[[2, 0, 1]], back[4:]])
    assert cases.rel_err(back.reshape(5, -1), ref.reshape(5, -1)) < 1e-13


# ------------------------------------------------------- linear advection P6
def test_linear_advection_closed_form():
    n, u, p, g = 32, 0.7, 1.0, 1.4
    x = (np.arange(n) + 0.5) / n
    r1 = 1.0 + 0.5 * np.sin(2 * np.pi * x) + 0.3 * (x > 0.6)
    rho = np.broadcast_to(r1[None, None, :], (2, 2, n)).copy()
    U = W.conserved(rho, np.full_like(rho, u), 0 * rho, 0 * rho, np.full_like(rho, p), g)
    prob = W.Problem("advect", 5, 5, (n, 2, 2), g, U)
    o = Oracle(prob)
    dt = 0.3 / n
    o.coarse_step(dt)
    Uo = o.download(5)
    xyz = o.coords(5)
    got = np.zeros(n)
    for ci in range(8):
        got[2 * xyz[:, 0] + (ci & 1)] = Uo[0, ci::8]
    lam = dt * n
    d = np.zeros(n)
    a = r1 - np.roll(r1, 1)
    b = np.roll(r1, -1) - r1
    d = np.where((a > 0) & (b > 0), np.minimum(a, b), np.where((a < 0) & (b < 0), np.maximum(a, b), 0.0))
    face = r1 + 0.5 * (1 - lam * u) * d         # rho_{L,i+1/2}
    expect = r1 - lam * u * (face - np.roll(face, 1))
    np.testing.assert_allclose(got, expect, rtol=1e-13, atol=0)


# ----------------------------------------------------------- CFL closed form
def test_cfl_uniform_closed_form():
    prob = W.uniform_state(8, rho=1.3, v=(0.3, -0.2, 0.1), p=0.7, gamma=1.4)
    o = Oracle(prob)
    c = math.sqrt(1.4 * 0.7 / 1.3)
    expect = 0.8 * (1 / 8) / (0.3 + 0.2 + 0.1 + 3 * c)
    assert abs(o.cfl_dt() - expect) <= 1e-15 * expect


# ------------------------------------------------- AMR equivalences (P7, P8)
def test_fully_refined_amr_equals_uniform_fine_bit_exact():
    fine = W.random_smooth(16, seed=31, mach=1.2)
    Uf = fine.U_base                           # (5, z, y, x)

    def fill(level, ijk):
        return Uf[:, ijk[:, 2], ijk[:, 1], ijk[:, 0]]
    amr = W.Problem("full", 3, 4, (8, 8, 8), fine.gamma, W.tree_mean(Uf), refine=W.REFINE_MASS,
                    refine_param=0.0, fill=fill)
    oa = Oracle(amr)
    assert oa.level_info(4)[0] == 512 and oa.level_info(3)[1] == 0
    of = Oracle(fine)
    for _ in range(3):
        dt = oa.cfl_dt()
        assert dt == 2.0 * of.cfl_dt()
        oa.coarse_step(dt)
        of.coarse_step(0.5 * dt)
        of.coarse_step(0.5 * dt)
    np.testing.assert_array_equal(dense_level(oa, 4), dense_level(of, 4))


def test_unrefined_amr_equals_uniform_coarse_bit_exact():
    base = W.random_smooth(8, seed=41)
    amr = W.Problem("unref", 3, 5, (8, 8, 8), base.gamma, base.U_base, refine=W.REFINE_MASS,
                    refine_param=1e30, fill=lambda l, ijk: np.zeros((5, len(ijk))))
    oa, ob = Oracle(amr), Oracle(base)
    assert oa.level_info(4)[0] == 0
    oa.advance(4)
    ob.advance(4)
    np.testing.assert_array_equal(oa.download(3), ob.download(3))


# ------------------------------------------------------ dense brute force P9
def run_dense_vs_oracle(prob, steps):
    o = Oracle(prob)
    nl = prob.level_max - prob.level_min + 1
    dense = DenseAMR(prob.nbase[0], nl, prob.gamma, prob.cfl, prob.bc)
    for k, l in enumerate(o.levels):
        n, _ = o.level_info(l)
        if n:
            dense.load_from_octs(k, o.coords(l), o.download(l))
    # the oracle's refinement map satisfies the neighbour rule
    for k in range(1, nl):
        ex = dense.exists[k]
        if not ex.any():
            continue
        par = dense.exists[k - 1]
        idx = np.argwhere(ex[0::2, 0::2, 0::2])   # refined parent cells at k-1
        n = par.shape[0]
        for (i, j, m) in idx:
            for di in (-1, 0, 1):
                for dj in (-1, 0, 1):
                    for dm in (-1, 0, 1):
                        q = np.array([i + di, j + dj, m + dm])
                        if prob.bc[0] == W.BC_PERIODIC:
                            q %= n
                        elif (q < 0).any() or (q >= n).any():
                            continue
                        assert par[tuple(q)]
    for s in range(steps):
        dt_o = o.cfl_dt()
        dt_d = dense.cfl_dt()
        assert abs(dt_o - dt_d) <= 1e-14 * dt_o
        o.coarse_step(dt_o)
        dense.advance(0, dt_o, 0)
    worst = 0.0
    for k, l in enumerate(o.levels):
        n, _ = o.level_info(l)
        if n:
            worst = max(worst, cases.rel_err(dense.to_octs(k, o.coords(l)), o.download(l)))
    return o, worst


@pytest.mark.parametrize("centre", [(0.06, 0.92, 0.5), (0.5, 0.5, 0.97)])
def test_dense_bruteforce_matches_octree_periodic(centre):
    prob = cases.amr_blob(centre=centre)
    o, worst = run_dense_vs_oracle(prob, 3)
    assert o.level_info(4)[0] > 0 and o.level_info(5)[0] > 0
    assert worst < 1e-13, worst


def test_dense_bruteforce_matches_octree_outflow():
    prob = cases.amr_blob(bc=(W.BC_OUTFLOW,) * 6, centre=(0.1, 0.5, 0.5), lshape=True)
    o, worst = run_dense_vs_oracle(prob, 3)
    assert o.level_info(4)[0] > 0
    assert worst < 1e-13, worst


# ------------------------------------------------------ refinement map P10
def test_refinement_map_step_field_gradient():
    # density 1 for x < 0.5, 2 for x >= 0.5 at level 3 (8^3, periodic): the
    # jumps sit between cells 3|4 and 7|0.  The central difference of a cell
    # next to a jump is +-0.5, so |g|/rho = 0.5 on the rho=1 side (cells 0 and
    # 3) and 0.25 on the rho=2 side (cells 4 and 7): theta = 0.3 flags exactly
    # the planes x = 0 and x = 3.
    def state(pos):
        rho = np.where(pos[:, 0] < 0.5, 1.0, 2.0)
        z = np.zeros(len(pos))
        return rho, z, z, z, np.ones(len(pos))
    prob = cases.analytic_problem("step", 3, 4, state, theta=0.3)
    o = Oracle(prob)
    keys, ref = o.mesh(3)
    xyz = o.coords(3)
    flagged = set()
    for oi in range(len(keys)):
        for ci in range(8):
            if ref[oi] & (1 << ci):
                flagged.add((2 * xyz[oi, 0] + (ci & 1), 2 * xyz[oi, 1] + ((ci >> 1) & 1),
                             2 * xyz[oi, 2] + ((ci >> 2) & 1)))
    expect = {(x, y, z) for x in (0, 3) for y in range(8) for z in range(8)}
    assert flagged == expect
    assert o.level_info(4)[0] == len(expect)


def test_refinement_mass_threshold_exact_power_of_eight():
    def state(pos):
        rho = np.where(pos[:, 0] < 0.5, 7.999999, 8.000001)
        z = np.zeros(len(pos))
        return rho, z, z, z, np.ones(len(pos))
    prob = cases.analytic_problem("mass", 3, 5, state, rho_thr=1.0)
    o = Oracle(prob)
    n4, _ = o.level_info(4)
    n5, _ = o.level_info(5)
    assert n4 > 0
    assert n5 > 0         # level 4 cells with rho 8.000001 > 1 * 8
    xyz5 = o.coords(5)
    assert (xyz5[:, 0] >= 8).all()   # only the x >= 0.5 half reaches level 5


# -------------------------------------------- smooth-flow order of accuracy
def acoustic_error(n, eps=1e-4, g=1.4):
    x = (np.arange(n) + 0.5) / n
    c = math.sqrt(g)
    s = np.sin(2 * np.pi * x)
    rho = np.broadcast_to((1 + eps * s)[None, None, :], (2, 2, n)).copy()
    u = np.broadcast_to((c * eps * s)[None, None, :], (2, 2, n)).copy()
    p = np.broadcast_to((1 + g * eps * s)[None, None, :], (2, 2, n)).copy()
    z = np.zeros_like(rho)
    U = W.conserved(rho, u, z, z, p, g)
    lvl = int(round(math.log2(n)))
    prob = W.Problem(f"acoustic{n}", lvl, lvl, (n, 2, 2), g, U)
    o = Oracle(prob)
    o.advance(100000, 1.0 / c)          # one period: the wave returns
    Uo = o.download(lvl)
    xyz = o.coords(lvl)
    got = np.zeros(n)
    for ci in range(8):
        got[2 * xyz[:, 0] + (ci & 1)] = Uo[0, ci::8]
    # exact cell averages of the linear wave after one period
    exact = 1 + eps * (np.cos(2 * np.pi * (x - 0.5 / n)) - np.cos(2 * np.pi * (x + 0.5 / n))) * n / (2 * np.pi)
    return np.abs(got - exact).mean() / eps


def test_acoustic_wave_second_order():
    e = [acoustic_error(n) for n in (32, 64, 128)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert orders[1] > 1.6, (e, orders)
