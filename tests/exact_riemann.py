"""Exact Riemann solver for the 1-D Euler equations of an ideal gas.

Follows Toro (2009), "Riemann Solvers and Numerical Methods for Fluid
Dynamics", 3rd ed., chapter 4: the pressure function f(p) = f_L(p) + f_R(p)
+ (u_R - u_L) (shock branch for p > p_K, rarefaction branch otherwise),
Newton-Raphson for the star pressure, and the self-similar sampling of the
solution at x/t.  Used only to pin the oracle (the Sod test).
"""
from __future__ import annotations

import math

import numpy as np


def _fK(p, rho, pK, g):
    """Toro (4.6)-(4.7): f_K and its derivative."""
    A = 2.0 / ((g + 1.0) * rho)
    B = (g - 1.0) / (g + 1.0) * pK
    c = math.sqrt(g * pK / rho)
    if p > pK:  # shock
        s = math.sqrt(A / (p + B))
        f = (p - pK) * s
        df = s * (1.0 - 0.5 * (p - pK) / (B + p))
    else:       # rarefaction
        f = 2.0 * c / (g - 1.0) * ((p / pK) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * c) * (p / pK) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, g, tol=1e-14):
    """Star pressure and velocity (Toro sec. 4.3)."""
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    # two-rarefaction guess (Toro 4.46), positive
    z = (g - 1.0) / (2.0 * g)
    p = ((cl + cr - 0.5 * (g - 1.0) * (ur - ul)) / (cl / pl ** z + cr / pr ** z)) ** (1.0 / z)
    for _ in range(100):
        fl, dfl = _fK(p, rl, pl, g)
        fr, dfr = _fK(p, rr, pr, g)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        if pn < 0:
            pn = tol
        if 2.0 * abs(pn - p) / (pn + p) < tol:
            p = pn
            break
        p = pn
    fl, _ = _fK(p, rl, pl, g)
    fr, _ = _fK(p, rr, pr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def star_densities(rl, pl, rr, pr, ps, g):
    def rho_star(rho, pK):
        if ps > pK:
            q = ps / pK
            gm = (g - 1.0) / (g + 1.0)
            return rho * (q + gm) / (gm * q + 1.0)
        return rho * (ps / pK) ** (1.0 / g)
    return rho_star(rl, pl), rho_star(rr, pr)


def sample(rl, ul, pl, rr, ur, pr, g, xi):
    """Solution (rho, u, p) at similarity coordinates xi = x/t (array)."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    rsl, rsr = star_densities(rl, pl, rr, pr, ps, g)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for i, s in enumerate(xi.ravel()):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                SL = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                w = (rl, ul, pl) if s <= SL else (rsl, us, ps)
            else:        # left rarefaction
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                shl, stl = ul - cl, us - csl
                if s <= shl:
                    w = (rl, ul, pl)
                elif s >= stl:
                    w = (rsl, us, ps)
                else:
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    w = (rl * (c / cl) ** (2 / (g - 1)), 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s),
                         pl * (c / cl) ** (2 * g / (g - 1)))
        else:        # right of contact
            if ps > pr:  # right shock
                SR = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                w = (rr, ur, pr) if s >= SR else (rsr, us, ps)
            else:
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                shr, str_ = ur + cr, us + csr
                if s >= shr:
                    w = (rr, ur, pr)
                elif s <= str_:
                    w = (rsr, us, ps)
                else:
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    w = (rr * (c / cr) ** (2 / (g - 1)), 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s),
                         pr * (c / cr) ** (2 * g / (g - 1)))
        rho.ravel()[i], u.ravel()[i], p.ravel()[i] = w
    return rho, u, p


def cell_average_density(rl, ul, pl, rr, ur, pr, g, x0, t, n, sub=64):
    """Exact cell averages of rho over n cells of [0,1] at time t."""
    xs = (np.arange(n * sub) + 0.5) / (n * sub)
    rho, _, _ = sample(rl, ul, pl, rr, ur, pr, g, (xs - x0) / t)
    return rho.reshape(n, sub).mean(axis=1)
