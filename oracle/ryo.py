"""ctypes driver of the FP64 CPU oracle (oracle/ryo.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark; never by the product path.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import build as _build


class RyoConfig(C.Structure):
    _fields_ = [("level_min", C.c_int32), ("level_max", C.c_int32), ("nbase", C.c_int32 * 3),
                ("boxlen", C.c_double), ("gamma", C.c_double), ("cfl", C.c_double),
                ("bc", C.c_int32 * 6), ("refine", C.c_int32), ("refine_param", C.c_double),
                ("rho_floor", C.c_double), ("p_floor", C.c_double), ("nscalar", C.c_int32)]


FILL_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_int32),
                      C.POINTER(C.c_double))

_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(_build.ensure_built())
        P = C.c_void_p
        L.ryo_create.argtypes = [C.POINTER(RyoConfig), C.POINTER(P)]
        L.ryo_destroy.argtypes = [P]
        L.ryo_amr_build.argtypes = [P, C.POINTER(C.c_double), FILL_FN, P]
        L.ryo_level_info.argtypes = [P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.ryo_get_mesh.argtypes = [P, C.c_int32, P, P]
        L.ryo_get_coords.argtypes = [P, C.c_int32, P]
        L.ryo_download.argtypes = [P, C.c_int32, P]
        L.ryo_upload.argtypes = [P, C.c_int32, P]
        L.ryo_cfl_dt.argtypes = [P, C.POINTER(C.c_double)]
        L.ryo_coarse_step.argtypes = [P, C.c_double]
        L.ryo_advance.argtypes = [P, C.c_int32, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
        L.ryo_conserved_totals.argtypes = [P, C.POINTER(C.c_double)]
        L.ryo_regrid.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.ryo_set_refine_param.argtypes = [P, C.c_double]
        L.ryo_floor_count.argtypes = [P]
        L.ryo_floor_count.restype = C.c_int64
        L.ryo_reset_floor_count.argtypes = [P]
        L.ryo_last_error.argtypes = [P]
        L.ryo_last_error.restype = C.c_char_p
        L.ryo_hilbert_key.argtypes = [C.c_int32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.ryo_hilbert_key.restype = C.c_uint64
        L.ryo_hllc.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32, C.c_double,
                               C.POINTER(C.c_double)]
        L.ryo_hllc_scalars.argtypes = [C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int32, C.c_int32,
                                       C.c_double, C.POINTER(C.c_double)]
        L.ryo_minmod.argtypes = [C.c_double, C.c_double]
        L.ryo_minmod.restype = C.c_double
        L.ryo_set_num_threads.argtypes = [C.c_int]
        L.ryo_num_threads.restype = C.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def make_fill(fill, nv=5):
    """Wrap a Python fill(level, ijk[n,3]) -> U[nv,n] as a C callback."""
    def cb(user, level, ncell, ijk, U):
        a = np.ctypeslib.as_array(ijk, shape=(ncell, 3))
        out = np.ctypeslib.as_array(U, shape=(nv, ncell))
        out[...] = fill(int(level), a.copy())
    return FILL_FN(cb)


class Oracle:
    """One oracle context built from a workloads.Problem."""

    def __init__(self, prob, threads: int | None = None):
        L = lib()
        if threads is not None:
            L.ryo_set_num_threads(int(threads))
        cfg = RyoConfig()
        cfg.level_min, cfg.level_max = prob.level_min, prob.level_max
        for a in range(3):
            cfg.nbase[a] = prob.nbase[a]
        cfg.boxlen, cfg.gamma, cfg.cfl = prob.boxlen, prob.gamma, prob.cfl
        for i in range(6):
            cfg.bc[i] = prob.bc[i]
        cfg.refine, cfg.refine_param = prob.refine, prob.refine_param
        cfg.rho_floor, cfg.p_floor = prob.rho_floor, prob.p_floor
        cfg.nscalar = prob.nscalar
        self.nv = 5 + prob.nscalar
        self.prob = prob
        self.ctx = C.c_void_p()
        self._check(L.ryo_create(C.byref(cfg), C.byref(self.ctx)), "create")
        base = prob.base_flat()
        nv = self.nv
        self._fill = make_fill(prob.fill if prob.fill else (lambda l, ijk: np.zeros((nv, len(ijk)))), nv)
        self._check(L.ryo_amr_build(self.ctx, base.ctypes.data_as(C.POINTER(C.c_double)), self._fill, None),
                    "amr_build")
        self.t = 0.0

    def _check(self, rc, what):
        if rc != 0:
            msg = lib().ryo_last_error(self.ctx).decode() if self.ctx else ""
            raise OracleError(f"ryo_{what} failed with {rc}: {msg}")

    def __del__(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            lib().ryo_destroy(self.ctx)
            self.ctx = C.c_void_p()

    @property
    def levels(self):
        return range(self.prob.level_min, self.prob.level_max + 1)

    def level_info(self, level):
        n, leaf = C.c_int64(), C.c_int64()
        self._check(lib().ryo_level_info(self.ctx, level, C.byref(n), C.byref(leaf)), "level_info")
        return n.value, leaf.value

    def mesh(self, level):
        n, _ = self.level_info(level)
        keys = np.zeros(n, np.uint64)
        ref = np.zeros(n, np.uint8)
        self._check(lib().ryo_get_mesh(self.ctx, level, keys.ctypes.data, ref.ctypes.data), "get_mesh")
        return keys, ref

    def coords(self, level):
        n, _ = self.level_info(level)
        xyz = np.zeros((n, 3), np.int32)
        self._check(lib().ryo_get_coords(self.ctx, level, xyz.ctypes.data), "get_coords")
        return xyz

    def download(self, level):
        n, _ = self.level_info(level)
        U = np.zeros((self.nv, 8 * n), np.float64)
        self._check(lib().ryo_download(self.ctx, level, U.ctypes.data), "download")
        return U

    def upload(self, level, U):
        U = np.ascontiguousarray(U, np.float64)
        self._check(lib().ryo_upload(self.ctx, level, U.ctypes.data), "upload")

    def cfl_dt(self):
        dt = C.c_double()
        self._check(lib().ryo_cfl_dt(self.ctx, C.byref(dt)), "cfl_dt")
        return dt.value

    def coarse_step(self, dt):
        self._check(lib().ryo_coarse_step(self.ctx, dt), "coarse_step")

    def advance(self, n_coarse, t_end=math.inf):
        t = C.c_double(self.t)
        nd = C.c_int32()
        self._check(lib().ryo_advance(self.ctx, n_coarse, t_end, C.byref(t), C.byref(nd)), "advance")
        self.t = t.value
        return nd.value

    def totals(self):
        tot = (C.c_double * self.nv)()
        self._check(lib().ryo_conserved_totals(self.ctx, tot), "conserved_totals")
        return np.array(tot[:])

    def floors(self):
        return lib().ryo_floor_count(self.ctx)

    def set_refine_param(self, value):
        self._check(lib().ryo_set_refine_param(self.ctx, value), "set_refine_param")

    def regrid(self):
        """Dynamic refinement between coarse steps: (octs created, destroyed)."""
        a, b = C.c_int64(), C.c_int64()
        self._check(lib().ryo_regrid(self.ctx, C.byref(a), C.byref(b)), "regrid")
        return a.value, b.value


def hilbert_key(bits, x, y, z):
    return lib().ryo_hilbert_key(bits, x, y, z)


def hllc(WL, WR, d, gamma):
    a = (C.c_double * 5)(*WL)
    b = (C.c_double * 5)(*WR)
    F = (C.c_double * 5)()
    lib().ryo_hllc(a, b, d, gamma, F)
    return np.array(F[:])


def hllc_scalars(WL, WR, d, gamma):
    """HLLC flux of (rho, u, v, w, p, s_1..s_k) states; len(WL) = 5 + k."""
    n = len(WL)
    a = (C.c_double * n)(*WL)
    b = (C.c_double * n)(*WR)
    F = (C.c_double * n)()
    lib().ryo_hllc_scalars(a, b, n - 5, d, gamma, F)
    return np.array(F[:])


def minmod(a, b):
    return lib().ryo_minmod(a, b)
