"""Seeded synthetic inputs shaped like the paper's workloads.

This module only generates initial conditions (density, velocity and
pressure fields turned into conserved variables, and point-value fill
functions for refined levels).  It holds none of the hydro method's
arithmetic; both the GPU library and the CPU oracle consume the identical
bytes it produces.

Recipes (seed = 1000 * config + field; field 0 = ln rho, 1..3 = v_x, v_y,
v_z; box b of the batched workload uses 5000 + 10 b + field):

* sod      -- 32^3, gamma 1.4, left state (rho, p) = (1, 1) for cells with
              centre x < 0.5, right state (0.125, 0.1), at rest, outflow.
* uniform  -- 128^3 periodic, gamma 5/3, p = 1, ln rho = white noise
              smoothed with a periodic Gaussian of sigma = 4 cells and
              renormalised to zero mean / unit variance; three velocity
              fields made the same way, scaled to rms Mach 1 against
              c0 = sqrt(gamma).
* twolevel -- the uniform generator at 128^3; the 64^3 base is the
              8-cell mean of the 128^3 conserved field, refined cells take
              the 128^3 values (gradient criterion, theta 0.70 or 0.1).
* zoom     -- levels 7-12, lognormal background (sigma 1.5), 64 Gaussian
              clumps in 8 clusters with peak contrast 1e3, p = rho, a
              smooth velocity field scaled to a maximum Mach number of 5,
              refined cells take point values (trilinear background plus
              analytic clumps), mass criterion.
* batch    -- 512 periodic boxes with sides in {16,24,32,40,48}, per box
              sigma ~ U(0.5, 1.5), rms Mach ~ U(0.5, 3), gamma 5/3, uniform
              temperature p = rho.
* uniform with scalars -- the uniform box plus passive scalars s_k =
              0.5 (1 + tanh g_k), g_k smoothed like ln rho (seed 1000 *
              config + 4 + k), stored as rho s_k.
* poisson  -- source of the cell-level Poisson equation on one uniform
              periodic level: the uniform generator's lognormal density
              (sigma_ln 1, smoothing 4 cells per 128 cells of box, seed
              6000), b = (mean rho - rho) dx^2 in units 4 pi G = 1, box 1.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import Callable, List, Optional

import numpy as np

BC_PERIODIC, BC_OUTFLOW = 0, 1
REFINE_NONE, REFINE_GRAD, REFINE_MASS = 0, 1, 2

FillFn = Callable[[int, np.ndarray], np.ndarray]


@dataclasses.dataclass
class Problem:
    """One hydro problem: mesh/config parameters plus initial data."""
    name: str
    level_min: int
    level_max: int
    nbase: tuple
    gamma: float
    U_base: np.ndarray            # (5 + nscalar, nz, ny, nx) float64, conserved variables
    boxlen: float = 1.0
    cfl: float = 0.8
    bc: tuple = (BC_PERIODIC,) * 6
    refine: int = REFINE_NONE
    refine_param: float = 0.0
    rho_floor: float = 1e-10
    p_floor: float = 1e-10
    fill: Optional[FillFn] = None  # (level, ijk[n,3] int32) -> U[5 + nscalar, n] float64
    t_end: float = math.inf
    n_steps: int = 10
    nscalar: int = 0              # passive scalars, conserved as rho*s after the 5 hydro planes

    def base_flat(self) -> np.ndarray:
        """U_base as 5 + nscalar contiguous planes, x fastest."""
        return np.ascontiguousarray(self.U_base.reshape(5 + self.nscalar, -1), dtype=np.float64)


def conserved(rho, vx, vy, vz, p, gamma):
    """Conserved variables (rho, rho v, E) of an ideal gas state."""
    E = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return np.stack([rho, rho * vx, rho * vy, rho * vz, E]).astype(np.float64)


def smooth_gaussian_field(n: int, seed: int, sigma_cells: float) -> np.ndarray:
    """Periodic white noise smoothed by a Gaussian of `sigma_cells`, then
    renormalised to zero mean and unit variance.  Array axes are (z, y, x)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    k = 2.0 * np.pi * np.fft.fftfreq(n)
    kz = k[:, None, None]
    ky = k[None, :, None]
    kx = k[None, None, : n // 2 + 1]
    filt = np.exp(-0.5 * sigma_cells ** 2 * (kx * kx + ky * ky + kz * kz))
    g = np.fft.irfftn(np.fft.rfftn(w) * filt, s=(n, n, n), axes=(0, 1, 2))
    g = g - g.mean()
    g = g / g.std()
    return g


def lognormal_fields(n, seed0, sigma_ln, mach_rms, gamma, smooth=4.0):
    rho = np.exp(sigma_ln * smooth_gaussian_field(n, seed0 + 0, smooth))
    v = [smooth_gaussian_field(n, seed0 + f, smooth) for f in (1, 2, 3)]
    c0 = math.sqrt(gamma)
    vrms = math.sqrt(float(np.mean(v[0] ** 2 + v[1] ** 2 + v[2] ** 2)))
    s = mach_rms * c0 / vrms
    p = np.ones_like(rho)
    return rho, v[0] * s, v[1] * s, v[2] * s, p


# ---------------------------------------------------------------------------
# config 1: Sod shock tube
# ---------------------------------------------------------------------------
def sod(n: int = 32, gamma: float = 1.4, t_end: float = 0.1) -> Problem:
    x = (np.arange(n) + 0.5) / n
    left = (x < 0.5)[None, None, :] * np.ones((n, n, 1), dtype=bool)
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    z = np.zeros_like(rho)
    U = conserved(rho, z, z, z, p, gamma)
    lvl = int(round(math.log2(n)))
    return Problem("sod", lvl, lvl, (n, n, n), gamma, U, bc=(BC_OUTFLOW,) * 6,
                   t_end=t_end, n_steps=1000)


# ---------------------------------------------------------------------------
# config 2: uniform periodic lognormal box
# ---------------------------------------------------------------------------
def uniform(n: int = 128, seed_cfg: int = 2, sigma_ln: float = 1.0, mach_rms: float = 1.0,
            gamma: float = 5.0 / 3.0, n_steps: int = 10, nscalar: int = 0) -> Problem:
    rho, vx, vy, vz, p = lognormal_fields(n, 1000 * seed_cfg, sigma_ln, mach_rms, gamma)
    U = conserved(rho, vx, vy, vz, p, gamma)
    if nscalar:
        U = np.concatenate([U, rho[None] * scalar_fields(n, 1000 * seed_cfg, nscalar)], axis=0)
    lvl = int(round(math.log2(n)))
    return Problem(f"uniform{n}" + (f"_s{nscalar}" if nscalar else ""), lvl, lvl, (n, n, n), gamma, U,
                   n_steps=n_steps, nscalar=nscalar)


def scalar_fields(n: int, seed0: int, nscalar: int) -> np.ndarray:
    """Passive scalars s_k in (0, 1): smoothed Gaussian fields (seeds seed0 +
    4 + k, sigma 4 cells) through 0.5 (1 + tanh); metallicity-like tracers."""
    return np.array([0.5 * (1.0 + np.tanh(smooth_gaussian_field(n, seed0 + 4 + k, 4.0))) for k in range(nscalar)])


# ---------------------------------------------------------------------------
# config 3: two-level AMR from a 128^3 field
# ---------------------------------------------------------------------------
def tree_mean(U: np.ndarray) -> np.ndarray:
    """8-cell mean of a (5, 2n, 2n, 2n) field -> (5, n, n, n)."""
    c = [U[:, iz::2, iy::2, ix::2] for iz in (0, 1) for iy in (0, 1) for ix in (0, 1)]
    return 0.125 * (((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7])))


def twolevel(n_fine: int = 128, theta: float = 0.70, gamma: float = 5.0 / 3.0,
             n_steps: int = 10) -> Problem:
    rho, vx, vy, vz, p = lognormal_fields(n_fine, 3000, 1.0, 1.0, gamma)
    Uf = conserved(rho, vx, vy, vz, p, gamma)
    Ub = tree_mean(Uf)
    lf = int(round(math.log2(n_fine)))

    def fill(level: int, ijk: np.ndarray) -> np.ndarray:
        assert level == lf
        return Uf[:, ijk[:, 2], ijk[:, 1], ijk[:, 0]]

    nb = n_fine // 2
    return Problem(f"twolevel{n_fine}_t{theta}", lf - 1, lf, (nb, nb, nb), gamma, Ub,
                   refine=REFINE_GRAD, refine_param=theta, fill=fill, n_steps=n_steps)


# ---------------------------------------------------------------------------
# config 4: zoom-shaped AMR
# ---------------------------------------------------------------------------
ZOOM_RHO_THR = 3.5     # mass criterion threshold at the base level (about 2M octs)
ZOOM_R_CLUMP = 0.012   # clump radius (box units)


class ZoomField:
    """Analytic density/velocity field of the zoom workload (point values)."""

    def __init__(self, n: int = 128, r_clump: float = ZOOM_R_CLUMP, gamma: float = 5.0 / 3.0,
                 mach_max: float = 5.0):
        self.n = n
        self.gamma = gamma
        self.rc = r_clump
        self.lnbg = 1.5 * smooth_gaussian_field(n, 4000, 4.0)
        vel = [smooth_gaussian_field(n, 4000 + f, 8.0) for f in (1, 2, 3)]
        vmax = float(np.sqrt(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2).max())
        s = mach_max * math.sqrt(gamma) / vmax
        self.vel = [v * s for v in vel]
        self.grids = np.stack([self.lnbg] + self.vel)   # (4, z, y, x)
        rng = np.random.default_rng(4004)
        centres = rng.random((8, 3))
        offs = rng.normal(0.0, 1.0 / 32.0, size=(8, 8, 3))
        self.clumps = np.mod(centres[:, None, :] + offs, 1.0).reshape(64, 3)

    def _trilinear(self, fields: np.ndarray, pos: np.ndarray) -> np.ndarray:
        """Periodic trilinear interpolation of cell-centred grids
        fields (k, n, n, n) at points pos (m, 3) -> (k, m)."""
        n = self.n
        flat = fields.reshape(fields.shape[0], -1)
        s = pos * n - 0.5                         # grid coordinates (cell centred)
        i0 = np.floor(s).astype(np.int64)
        f = s - i0
        out = np.zeros((fields.shape[0], pos.shape[0]))
        for dz in (0, 1):
            wz = f[:, 2] if dz else 1.0 - f[:, 2]
            iz = (i0[:, 2] + dz) % n
            for dy in (0, 1):
                wy = f[:, 1] if dy else 1.0 - f[:, 1]
                iy = (i0[:, 1] + dy) % n
                wzy = wz * wy
                base = (iz * n + iy) * n
                for dx in (0, 1):
                    wx = f[:, 0] if dx else 1.0 - f[:, 0]
                    ix = (i0[:, 0] + dx) % n
                    out += (wzy * wx) * flat[:, base + ix]
        return out

    def values(self, level: int, ijk: np.ndarray, base_level: int = 7) -> np.ndarray:
        ncell = self.n << (level - base_level)
        pos = (ijk.astype(np.float64) + 0.5) / ncell
        g = self._trilinear(self.grids, pos)
        rho_bg = np.exp(g[0])
        boost = self._clump_sum(pos)
        rho = rho_bg * (1.0 + 1.0e3 * boost)
        return conserved(rho, g[1], g[2], g[3], rho.copy(), self.gamma)

    def _clump_sum(self, pos: np.ndarray) -> np.ndarray:
        """sum_k exp(-r_k^2 / (2 r_c^2)) over the clumps, in clump order,
        truncated at r^2 = 80 r_c^2 (periodic minimum-image distance).
        Points are binned on a coarse grid so each clump only visits the
        bins it can reach; the value of each point is unchanged by that."""
        nb = max(1, int(1.0 / (math.sqrt(80.0) * self.rc)))
        b = np.minimum((pos * nb).astype(np.int64), nb - 1)
        bid = (b[:, 2] * nb + b[:, 1]) * nb + b[:, 0]
        order = np.argsort(bid, kind="stable")
        sorted_bid = bid[order]
        starts = np.searchsorted(sorted_bid, np.arange(nb ** 3 + 1))
        boost = np.zeros(pos.shape[0])
        inv2 = 1.0 / (2.0 * self.rc * self.rc)
        cut = 80.0 * self.rc * self.rc
        for c in self.clumps:
            cb = np.minimum((c * nb).astype(np.int64), nb - 1)
            near = set()
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        near.add(((((cb[2] + dz) % nb) * nb + (cb[1] + dy) % nb) * nb + (cb[0] + dx) % nb))
            idx = np.concatenate([order[starts[k]:starts[k + 1]] for k in sorted(near)])
            if idx.size == 0:
                continue
            d = pos[idx] - c
            d -= np.round(d)
            r2 = np.einsum("ij,ij->i", d, d)
            m = r2 < cut
            boost[idx[m]] += np.exp(-r2[m] * inv2)
        return boost


def zoom(level_min: int = 7, level_max: int = 12, rho_thr: float = ZOOM_RHO_THR,
         r_clump: float = ZOOM_R_CLUMP, n_steps: int = 10) -> Problem:
    n = 1 << level_min
    zf = ZoomField(n, r_clump)
    idx = np.indices((n, n, n))  # (3, z, y, x)
    ijk = np.stack([idx[2].ravel(), idx[1].ravel(), idx[0].ravel()], axis=1).astype(np.int32)
    Ub = zf.values(level_min, ijk, level_min).reshape(5, n, n, n)

    cache = {}

    def fill(level: int, ijk: np.ndarray) -> np.ndarray:
        # both consumers (GPU library and oracle) request the same cells in
        # the same order; keep the last answer per level to skip recomputing
        key = (level, ijk.shape[0], hashlib.blake2b(ijk.tobytes(), digest_size=16).hexdigest())
        if key not in cache:
            cache.clear() if len(cache) > 8 else None
            cache[key] = zf.values(level, ijk, level_min)
        return cache[key]

    return Problem(f"zoom{level_min}-{level_max}", level_min, level_max, (n, n, n), 5.0 / 3.0, Ub,
                   refine=REFINE_MASS, refine_param=rho_thr, fill=fill, n_steps=n_steps)


# ---------------------------------------------------------------------------
# config 5: batched uneven periodic boxes
# ---------------------------------------------------------------------------
BATCH_SIDES = (16, 24, 32, 40, 48)


def batch_box(b: int, side: int, sigma_ln: float, mach: float, gamma: float = 5.0 / 3.0) -> Problem:
    # uniform temperature (p = rho): the rms Mach number is relative to the
    # one sound speed sqrt(gamma) everywhere in the box
    rho, vx, vy, vz, _ = lognormal_fields(side, 5000 + 10 * b, sigma_ln, mach, gamma)
    U = conserved(rho, vx, vy, vz, rho.copy(), gamma)
    return Problem(f"box{b}", 1, 1, (side, side, side), gamma, U, n_steps=20)


def batch(nbox: int = 512) -> List[Problem]:
    rng = np.random.default_rng(5000)
    sides = rng.choice(np.array(BATCH_SIDES), size=nbox)
    sig = rng.uniform(0.5, 1.5, size=nbox)
    mach = rng.uniform(0.5, 3.0, size=nbox)
    return [batch_box(b, int(sides[b]), float(sig[b]), float(mach[b])) for b in range(nbox)]


# ---------------------------------------------------------------------------
# small cases used by the tests
# ---------------------------------------------------------------------------
def uniform_state(n=8, rho=1.3, v=(0.3, -0.2, 0.1), p=0.7, gamma=1.4, bc=(BC_PERIODIC,) * 6) -> Problem:
    shape = (n, n, n)
    U = conserved(np.full(shape, rho), np.full(shape, v[0]), np.full(shape, v[1]),
                  np.full(shape, v[2]), np.full(shape, p), gamma)
    lvl = int(round(math.log2(n)))
    return Problem("uniform_state", lvl, lvl, shape, gamma, U, bc=bc)


def random_smooth(n=16, seed=7, sigma_ln=0.5, mach=0.8, gamma=1.4, smooth=2.0) -> Problem:
    rho, vx, vy, vz, p = lognormal_fields(n, seed, sigma_ln, mach, gamma, smooth)
    p = p * np.exp(0.3 * smooth_gaussian_field(n, seed + 7, smooth))
    U = conserved(rho, vx, vy, vz, p, gamma)
    lvl = int(round(math.log2(n)))
    return Problem(f"random{n}", lvl, lvl, (n, n, n), gamma, U)


# ---------------------------------------------------------------------------
# Poisson solver workload: gravity source of a lognormal density on one
# uniform periodic level
# ---------------------------------------------------------------------------
def poisson_source(n: int = 256, seed: int = 6000, sigma_ln: float = 1.0) -> np.ndarray:
    """b[z, y, x] = (mean(rho) - rho) / n^2 (zero sum, as a periodic problem needs)."""
    rho = np.exp(sigma_ln * smooth_gaussian_field(n, seed, 4.0 * n / 128.0))
    b = (rho.mean() - rho) / float(n * n)
    return b - b.mean()
