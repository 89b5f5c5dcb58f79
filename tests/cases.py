"""Small analytic test problems shared by the oracle pins and GPU parity tests.

Everything here is input generation (initial conditions and refinement
thresholds); none of the hydro method's arithmetic lives here.
"""
from __future__ import annotations

import math

import numpy as np

import workloads as W


def cell_centres(level: int, ijk: np.ndarray, n_at_level: int) -> np.ndarray:
    return (ijk.astype(np.float64) + 0.5) / n_at_level


def analytic_problem(name, level_min, level_max, state_fn, rho_thr=None, theta=None, gamma=1.4,
                     bc=(W.BC_PERIODIC,) * 6, cfl=0.8):
    """Problem whose every level takes point values state_fn(pos[n,3]) ->
    (rho, vx, vy, vz, p) at cell centres; refinement by mass threshold or
    gradient criterion."""
    n0 = 1 << level_min

    def values(level, ijk):
        pos = cell_centres(level, ijk, 1 << level)
        rho, vx, vy, vz, p = state_fn(pos)
        return W.conserved(rho, vx, vy, vz, p, gamma)

    idx = np.indices((n0, n0, n0))
    ijk = np.stack([idx[2].ravel(), idx[1].ravel(), idx[0].ravel()], axis=1).astype(np.int32)
    Ub = values(level_min, ijk).reshape(5, n0, n0, n0)
    refine, param = W.REFINE_NONE, 0.0
    if rho_thr is not None:
        refine, param = W.REFINE_MASS, rho_thr
    elif theta is not None:
        refine, param = W.REFINE_GRAD, theta
    return W.Problem(name, level_min, level_max, (n0, n0, n0), gamma, Ub, cfl=cfl, bc=bc,
                     refine=refine, refine_param=param, fill=values)


def _pdist(pos, c):
    d = pos - np.asarray(c)
    return d - np.round(d)


def blob_state(pos, centre=(0.06, 0.92, 0.5), amp=60.0, width=0.08, mach=0.9, lshape=True):
    """Density blob (wrapping across periodic faces) plus an L-shaped slab,
    smooth swirling velocity, smoothly varying pressure."""
    d = _pdist(pos, centre)
    r2 = (d * d).sum(axis=1)
    rho = 1.0 + amp * np.exp(-r2 / (2 * width * width))
    if lshape:
        x, y, z = pos[:, 0], pos[:, 1], pos[:, 2]
        inz = (z > 0.3) & (z < 0.7)
        arm1 = (x > 0.25) & (x < 0.75) & (y > 0.25) & (y < 0.40)
        arm2 = (x > 0.25) & (x < 0.40) & (y > 0.25) & (y < 0.75)
        rho = rho + 4.0 * (inz & (arm1 | arm2))
    tp = 2 * math.pi
    vx = mach * np.sin(tp * pos[:, 1]) * np.cos(tp * pos[:, 2])
    vy = mach * np.sin(tp * pos[:, 2] + 0.3) * np.cos(tp * pos[:, 0])
    vz = 0.5 * mach * np.sin(tp * pos[:, 0] + 0.7)
    p = 1.0 + 0.3 * np.cos(tp * (pos[:, 0] + 2 * pos[:, 1])) * np.sin(tp * pos[:, 2])
    return rho, vx, vy, vz, p


def amr_blob(level_min=3, level_max=5, rho_thr=1.5, bc=(W.BC_PERIODIC,) * 6, **kw):
    return analytic_problem(f"blob{level_min}-{level_max}", level_min, level_max,
                            lambda pos: blob_state(pos, **kw), rho_thr=rho_thr, bc=bc)


def noncubic_blob(bc=(W.BC_PERIODIC,) * 6, level_min=3, level_max=5, nbase=(8, 16, 12), gamma=1.4):
    """AMR blob on a box of different cell counts per axis (cubic cells,
    dx = 1 / nbase[0] at the base level), refined by the mass threshold."""
    def values(level, ijk):
        n = nbase[0] << (level - level_min)
        pos = (ijk.astype(np.float64) + 0.5) / n
        rho, vx, vy, vz, p = blob_state(pos, centre=(0.3, 1.4, 0.9), lshape=False)
        return W.conserved(rho, vx, vy, vz, p, gamma)

    idx = np.indices((nbase[2], nbase[1], nbase[0]))
    ijk = np.stack([idx[2].ravel(), idx[1].ravel(), idx[0].ravel()], axis=1).astype(np.int32)
    Ub = values(level_min, ijk).reshape(5, nbase[2], nbase[1], nbase[0])
    return W.Problem("ncblob", level_min, level_max, tuple(nbase), gamma, Ub, bc=bc, refine=W.REFINE_MASS,
                     refine_param=1.5, fill=values)


def rel_err(a, b, floor_frac=1e-3):
    """Per-variable relative error |a-b| / max(|b|, floor_frac * max|b_v|)."""
    a = np.asarray(a)
    b = np.asarray(b)
    scale = np.maximum(np.abs(b), floor_frac * np.abs(b).max(axis=-1, keepdims=True))
    scale = np.where(scale == 0, 1.0, scale)
    return float((np.abs(a - b) / scale).max())


def scalar_profiles(pos):
    """Four passive-scalar profiles: smooth, a step (exercises the limiter),
    a constant and a smooth one varying along z."""
    tp = 2 * math.pi
    return [0.5 + 0.4 * np.sin(tp * pos[:, 0]) * np.cos(tp * pos[:, 1]),
            np.where(pos[:, 0] + 0.3 * pos[:, 2] > 0.55, 0.9, 0.1),
            np.full(len(pos), 0.3),
            0.2 + 0.1 * np.cos(tp * pos[:, 2] + 0.4)]


def with_scalars(prob, nscalar, profiles=scalar_profiles):
    """A copy of a cubic-box problem with `nscalar` passive scalars appended
    (conserved rho*s, s from `profiles` at cell centres on every level)."""
    import dataclasses
    n0 = prob.nbase[0]

    def scal(level_cells, ijk, rho):
        pos = cell_centres(0, ijk, level_cells)
        s = profiles(pos)[:nscalar]
        return [rho * sk for sk in s]

    idx = np.indices(prob.U_base.shape[1:])
    ijk = np.stack([idx[2].ravel(), idx[1].ravel(), idx[0].ravel()], axis=1).astype(np.int32)
    rho0 = prob.U_base[0].ravel()
    extra = np.array(scal(n0, ijk, rho0)).reshape((nscalar,) + prob.U_base.shape[1:])
    Ub = np.concatenate([prob.U_base[:5], extra], axis=0)
    fill = None
    if prob.fill is not None:
        base_fill = prob.fill

        def fill(level, ijk):
            U = base_fill(level, ijk)
            cells = n0 << (level - prob.level_min)
            return np.concatenate([U[:5], np.array(scal(cells, ijk, U[0]))], axis=0)
    return dataclasses.replace(prob, name=prob.name + f"_s{nscalar}", U_base=Ub, fill=fill, nscalar=nscalar)


def leaf_mask(refined_bytes):
    """Per-cell leaf mask (8 cells per oct, bit c of the oct's byte = cell c
    refined)."""
    bits = np.unpackbits(np.asarray(refined_bytes, np.uint8)[:, None], axis=1, bitorder="little")
    return ~bits.astype(bool).reshape(-1)


def form_errors(levels_a, levels_b, gamma):
    """Errors of state a against the reference state b over the leaf cells
    of every level.  levels_* are lists of (U[nv, 8 n_oct], refined bytes,
    cell volume), the two lists on the same mesh.  Returns the volume-
    weighted relative L1 errors of density and pressure and the largest
    relative density and pressure errors."""
    def rho_p(U, m):
        r = U[0][m]
        p = (gamma - 1.0) * (U[4][m] - 0.5 * (U[1][m] ** 2 + U[2][m] ** 2 + U[3][m] ** 2) / r)
        return r, p

    l1r = l1p = nr = np_ = 0.0
    mr = mp = 0.0
    for (Ua, ra, va), (Ub, rb, vb) in zip(levels_a, levels_b):
        np.testing.assert_array_equal(ra, rb)
        m = leaf_mask(rb)
        a_r, a_p = rho_p(Ua, m)
        b_r, b_p = rho_p(Ub, m)
        l1r += np.abs(a_r - b_r).sum() * vb
        l1p += np.abs(a_p - b_p).sum() * vb
        nr += np.abs(b_r).sum() * vb
        np_ += np.abs(b_p).sum() * vb
        if len(b_r):
            mr = max(mr, float(np.max(np.abs(a_r - b_r) / np.abs(b_r))))
            mp = max(mp, float(np.max(np.abs(a_p - b_p) / np.abs(b_p))))
    return {"l1_rho_rel": float(l1r / nr), "l1_p_rel": float(l1p / np_), "max_rho_rel": mr, "max_p_rel": mp}


def level_states(h):
    """(U, refined bytes, cell volume) of every non-empty level of a GPU or
    oracle context."""
    out = []
    for k, lv in enumerate(h.levels):
        n, _ = h.level_info(lv)
        if n == 0:
            continue
        _, ref = h.mesh(lv)
        vol = (h.prob.boxlen / (h.prob.nbase[0] << k)) ** 3
        out.append((h.download(lv), ref, vol))
    return out
