"""Dense, level-by-level numpy implementation of the octree hydro step.

An independent re-implementation used ONLY to pin the octree oracle on tiny
meshes: every level is a dense periodic/outflow array with an "exists" mask
instead of a Hilbert-ordered oct list, ghosts are computed for whole levels
at once, coarse-fine registers are read straight out of the fine level's
face-flux arrays, and the HLLC star flux is written in Toro's (2009, sec.
10.4.2) alternative form F*_K = [S*(S_K U_K - F_K) + S_K p*_K D*]/(S_K - S*),
which is algebraically identical to F_K + S_K (U*_K - U_K) but rounds
differently, so an error in either form shows up as a mismatch.

Scheme (identical definitions to the oracle, written from the same textbook
sources): floors on rho and p; MinMod-limited undivided slopes of the
primitive variables; the unsplit half-step primitive predictor with
h = lambda/2; face states W~ +- D/2; HLLC with Davis wave speeds; the
conservative update; coarse-fine ghosts by MinMod-limited linear
interpolation of the covering coarse cell's conserved variables; fine-first
subcycling with Fbar = (q_1 + q_2)/8 and q_s the ordered sum of the four
fine-face fluxes; refined cells set to the mean of their children.
"""
from __future__ import annotations

import math

import numpy as np

BC_PERIODIC = 0


def minmod(a, b):
    return np.where((a > 0) & (b > 0), np.minimum(a, b),
                    np.where((a < 0) & (b < 0), np.maximum(a, b), 0.0))


class DenseAMR:
    def __init__(self, nbase, nlev, gamma, cfl, bc, boxlen=1.0, rho_floor=1e-10, p_floor=1e-10):
        self.nb = nbase
        self.L = nlev
        self.g = gamma
        self.cfl = cfl
        self.bc = bc
        self.boxlen = boxlen
        self.rf, self.pf = rho_floor, p_floor
        self.N = [nbase * (1 << k) for k in range(nlev)]
        self.exists = [np.zeros((n, n, n), bool) for n in self.N]
        self.U = [np.zeros((5, n, n, n)) for n in self.N]
        self.exists[0][...] = True
        self.fine_faces = [[None, None] for _ in range(nlev)]  # [level][substep] -> list of 3 arrays

    # ---------------------------------------------------------------- mesh
    def refined(self, k):
        if k + 1 >= self.L:
            return np.zeros_like(self.exists[k])
        return self.exists[k + 1][0::2, 0::2, 0::2].copy()

    def leaf(self, k):
        return self.exists[k] & ~self.refined(k)

    def dx(self, k):
        return self.boxlen / self.N[k]

    # ------------------------------------------------------------- helpers
    def _idx(self, n, pad, axis):
        i = np.arange(-pad, n + pad)
        if self.bc[2 * axis] == BC_PERIODIC:
            return i % n
        return np.clip(i, 0, n - 1)

    def pad(self, A, p):
        """Pad spatial axes (1,2,3) of A by p cells with the boundary rule."""
        n = A.shape[1]
        for ax in range(3):
            A = np.take(A, self._idx(n, p, ax), axis=1 + ax)
        return A

    def cover(self, k):
        """Finest existing value covering each position of level k."""
        C = self.U[0].copy()
        for j in range(1, k + 1):
            up = C.repeat(2, 1).repeat(2, 2).repeat(2, 3)
            C = np.where(self.exists[j][None], self.U[j], up)
        return C

    def resolved(self, k):
        """Level-k values: existing cells, else ghosts interpolated from k-1."""
        if k == 0:
            return self.U[0].copy()
        C = self.cover(k - 1)
        Cp = self.pad(C, 1)
        ctr = Cp[:, 1:-1, 1:-1, 1:-1]
        slopes = []
        for d in range(3):
            lo = [slice(None), slice(1, -1), slice(1, -1), slice(1, -1)]
            hi = list(lo)
            lo[1 + d] = slice(0, -2)
            hi[1 + d] = slice(2, None)
            slopes.append(minmod(ctr - Cp[tuple(lo)], Cp[tuple(hi)] - ctr))
        n = self.N[k]
        G = np.empty((5, n, n, n))
        for ix in (0, 1):
            for iy in (0, 1):
                for iz in (0, 1):
                    sx, sy, sz = (1.0 if ix else -1.0), (1.0 if iy else -1.0), (1.0 if iz else -1.0)
                    G[:, ix::2, iy::2, iz::2] = ctr + (sx * 0.25 * slopes[0] + sy * 0.25 * slopes[1]
                                                       + sz * 0.25 * slopes[2])
        return np.where(self.exists[k][None], self.U[k], G)

    def prim(self, V):
        rho = np.maximum(V[0], self.rf)
        ke = 0.5 * (V[1] * V[1] + V[2] * V[2] + V[3] * V[3]) / rho
        p = np.maximum((self.g - 1.0) * (V[4] - ke), self.pf)
        return np.stack([rho, V[1] / rho, V[2] / rho, V[3] / rho, p])

    def hllc(self, WL, WR, d):
        g = self.g
        t1, t2 = [a for a in range(3) if a != d]
        rl, ul, al, bl, pl = WL[0], WL[1 + d], WL[1 + t1], WL[1 + t2], WL[4]
        rr, ur, ar, br, pr = WR[0], WR[1 + d], WR[1 + t1], WR[1 + t2], WR[4]
        cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
        SL = np.minimum(ul - cl, ur - cr)
        SR = np.maximum(ul + cl, ur + cr)
        El = pl / (g - 1.0) + 0.5 * rl * (ul * ul + al * al + bl * bl)
        Er = pr / (g - 1.0) + 0.5 * rr * (ur * ur + ar * ar + br * br)
        Ss = (pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur)) / (rl * (SL - ul) - rr * (SR - ur))
        UL = np.stack([rl, rl * ul, rl * al, rl * bl, El])
        UR = np.stack([rr, rr * ur, rr * ar, rr * br, Er])
        FL = np.stack([rl * ul, rl * ul * ul + pl, rl * ul * al, rl * ul * bl, (El + pl) * ul])
        FR = np.stack([rr * ur, rr * ur * ur + pr, rr * ur * ar, rr * ur * br, (Er + pr) * ur])
        Dst = np.stack([np.zeros_like(Ss), np.ones_like(Ss), np.zeros_like(Ss), np.zeros_like(Ss), Ss])
        psl = pl + rl * (SL - ul) * (Ss - ul)
        psr = pr + rr * (SR - ur) * (Ss - ur)
        with np.errstate(all="ignore"):
            FsL = (Ss * (SL * UL - FL) + SL * psl * Dst) / (SL - Ss)
            FsR = (Ss * (SR * UR - FR) + SR * psr * Dst) / (SR - Ss)
        F = np.where(SL >= 0, FL, np.where(Ss >= 0, FsL, np.where(SR > 0, FsR, FR)))
        out = np.empty_like(F)
        out[0], out[1 + d], out[1 + t1], out[1 + t2], out[4] = F[0], F[1], F[2], F[3], F[4]
        return out

    # --------------------------------------------------------------- fluxes
    def face_fluxes(self, k, lam):
        """F[d][p] = flux through the face between p and p+e_d, for p in
        [-1, N-1] along d (array index p+1), other axes 0..N-1."""
        n = self.N[k]
        h = 0.5 * lam
        V = self.pad(self.resolved(k), 2)          # indices -2..n+1
        W = self.prim(V)
        g = self.g
        D = []
        for d in range(3):
            lo = [slice(None)] + [slice(1, -1)] * 3
            hi = list(lo)
            ctr = W[tuple(lo)]
            lo[1 + d] = slice(0, -2)
            hi[1 + d] = slice(2, None)
            D.append(minmod(ctr - W[tuple(lo)], W[tuple(hi)] - ctr))
        W0 = W[:, 1:-1, 1:-1, 1:-1]                 # indices -1..n
        r, u, v, w, p = W0
        Dx, Dy, Dz = D
        Wt = np.stack([
            r - h * (u * Dx[0] + r * Dx[1] + v * Dy[0] + r * Dy[2] + w * Dz[0] + r * Dz[3]),
            u - h * (u * Dx[1] + v * Dy[1] + w * Dz[1] + Dx[4] / r),
            v - h * (u * Dx[2] + v * Dy[2] + w * Dz[2] + Dy[4] / r),
            w - h * (u * Dx[3] + v * Dy[3] + w * Dz[3] + Dz[4] / r),
            p - h * (u * Dx[4] + v * Dy[4] + w * Dz[4] + g * p * (Dx[1] + Dy[2] + Dz[3])),
        ])
        F = []
        for d in range(3):
            a = [slice(None)] + [slice(1, n + 1)] * 3
            b = list(a)
            a[1 + d] = slice(0, n + 1)
            b[1 + d] = slice(1, n + 2)
            WL = Wt[tuple(a)] + 0.5 * D[d][tuple(a)]
            WR = Wt[tuple(b)] - 0.5 * D[d][tuple(b)]
            WL[0] = np.maximum(WL[0], self.rf)
            WR[0] = np.maximum(WR[0], self.rf)
            WL[4] = np.maximum(WL[4], self.pf)
            WR[4] = np.maximum(WR[4], self.pf)
            F.append(self.hllc(WL, WR, d))
        return F

    def register_flux(self, k, d):
        """Fbar on every level-k face along d from level k+1's stored fluxes,
        indexed like face_fluxes (face p between p and p+1, p in -1..N-1)."""
        Ff = [self.fine_faces[k + 1][s][d] for s in (0, 1)]
        nk = self.N[k]
        q = []
        for s in (0, 1):
            A = Ff[s]                                # fine face index p+1, p in -1..2nk-1
            t = [a for a in range(3) if a != d]
            sel = [slice(None)] * 4
            sel[1 + d] = slice(0, 2 * nk + 1, 2)     # fine p = 2P+1 -> index 2P+2; P=-1..nk-1 -> 0..2nk
            B = A[tuple(sel)]                        # coarse face index P+1

            def part(o1, o2):
                s_ = [slice(None)] * 4
                s_[1 + t[0]] = slice(o1, None, 2)
                s_[1 + t[1]] = slice(o2, None, 2)
                return B[tuple(s_)]
            q.append((part(0, 0) + part(1, 0)) + (part(0, 1) + part(1, 1)))
        return 0.125 * (q[0] + q[1])

    def update(self, k, lam, substep):
        n = self.N[k]
        F = self.face_fluxes(k, lam)
        self.fine_faces[k][substep] = [f.copy() for f in F]
        if k + 1 < self.L and self.exists[k + 1].any():
            ref = self.refined(k)
            for d in range(3):
                # refined flag of the lower (a) and upper (b) cell of each face
                R = self.pad(ref[None].astype(np.float64), 1)[0] > 0.5
                a = [slice(1, n + 1)] * 3
                b = list(a)
                a[d] = slice(0, n + 1)
                b[d] = slice(1, n + 2)
                ra, rb = R[tuple(a)], R[tuple(b)]
                mask = ra ^ rb          # one side refined, the other a leaf
                Fbar = self.register_flux(k, d)
                F[d] = np.where(mask[None], Fbar, F[d])
        acc = None
        for d in range(3):
            lo = [slice(None)] + [slice(None)] * 3
            hi = list(lo)
            lo[1 + d] = slice(0, n)
            hi[1 + d] = slice(1, n + 1)
            term = F[d][tuple(lo)] - F[d][tuple(hi)]
            acc = term if acc is None else acc + term
        Un = self.U[k] + lam * acc
        leaf = self.leaf(k)
        Un = np.where(leaf[None], Un, self.U[k])
        return Un

    def restrict(self, k, Un):
        Uf = self.U[k + 1]
        c = [Uf[:, ix::2, iy::2, iz::2] for iz in (0, 1) for iy in (0, 1) for ix in (0, 1)]
        mean = 0.125 * (((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7])))
        ref = self.refined(k)
        return np.where(ref[None], mean, Un)

    def advance(self, k, dt, substep):
        if k + 1 < self.L and self.exists[k + 1].any():
            self.advance(k + 1, 0.5 * dt, 0)
            self.advance(k + 1, 0.5 * dt, 1)
        lam = dt / self.dx(k)
        Un = self.update(k, lam, substep)
        if k + 1 < self.L and self.exists[k + 1].any():
            Un = self.restrict(k, Un)
        self.U[k] = Un

    def cfl_dt(self):
        best = math.inf
        for k in range(self.L):
            lf = self.leaf(k)
            if not lf.any():
                continue
            W = self.prim(self.U[k])
            c = np.sqrt(self.g * W[4] / W[0])
            s = np.abs(W[1]) + np.abs(W[2]) + np.abs(W[3]) + 3.0 * c
            smax = s[lf].max()
            best = min(best, math.ldexp(self.cfl * self.dx(k) / smax, k))
        return best

    # -------------------------------------------------- oracle (de)serialise
    def load_from_octs(self, k, coords, U):
        """coords: (n,3) oct coords; U: (5, 8n) in in-oct cell order."""
        for ci in range(8):
            ix, iy, iz = ci & 1, (ci >> 1) & 1, (ci >> 2) & 1
            X = 2 * coords[:, 0] + ix
            Y = 2 * coords[:, 1] + iy
            Z = 2 * coords[:, 2] + iz
            self.exists[k][X, Y, Z] = True
            self.U[k][:, X, Y, Z] = U[:, ci::8]

    def to_octs(self, k, coords):
        n = coords.shape[0]
        out = np.zeros((5, 8 * n))
        for ci in range(8):
            ix, iy, iz = ci & 1, (ci >> 1) & 1, (ci >> 2) & 1
            out[:, ci::8] = self.U[k][:, 2 * coords[:, 0] + ix, 2 * coords[:, 1] + iy, 2 * coords[:, 2] + iz]
        return out
