"""ctypes driver of the FP64 CPU oracle of the uniform-level Poisson solvers
(oracle/poisson.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark; never by the product path.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from .ryo import lib as _ryo_lib

PERIODIC, DIRICHLET = 0, 1
PC_NONE, PC_STENCIL7 = 0, 1

_done = False


class PPCGState(C.Structure):
    _fields_ = [(k, C.POINTER(C.c_double)) for k in ("x", "r", "u", "w", "z", "q", "s", "p")] + [
        ("alpha_prev", C.c_double), ("gamma_prev", C.c_double), ("i", C.c_int32)]


def lib():
    global _done
    L = _ryo_lib()
    if not _done:
        P = C.c_void_p
        N3 = C.POINTER(C.c_int32)
        L.ryo_poisson_apply_A.argtypes = [N3, C.c_int32, P, P]
        L.ryo_poisson_apply_Minv.argtypes = [N3, C.c_int32, C.c_int32, P, P]
        for f in (L.ryo_pcg, L.ryo_ppcg):
            f.argtypes = [N3, C.c_int32, C.c_int32, P, P, C.c_double, C.c_int32, P]
            f.restype = C.c_int32
        L.ryo_ppcg_init.argtypes = [N3, C.c_int32, C.c_int32, P, P, C.POINTER(PPCGState)]
        L.ryo_ppcg_dots.argtypes = [N3, C.POINTER(PPCGState), C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ryo_ppcg_step.argtypes = [N3, C.c_int32, C.c_int32, C.POINTER(PPCGState), C.c_double, C.c_double]
        _done = True
    return L


def _n3(shape):
    """(n0, n1, n2) with x fastest from a numpy array of shape (n2, n1, n0)."""
    return (C.c_int32 * 3)(shape[2], shape[1], shape[0])


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def apply_A(x, bc=PERIODIC):
    """A x for a grid array x[k, j, i] (x fastest)."""
    x = _f64(x)
    y = np.empty_like(x)
    lib().ryo_poisson_apply_A(_n3(x.shape), bc, _ptr(x), _ptr(y))
    return y


def apply_Minv(x, bc=PERIODIC, pc=PC_STENCIL7):
    x = _f64(x)
    y = np.empty_like(x)
    lib().ryo_poisson_apply_Minv(_n3(x.shape), bc, pc, _ptr(x), _ptr(y))
    return y


def _solve(fn, b, bc, pc, eps, max_iter, x0):
    b = _f64(b)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    hist = np.zeros(max_iter + 1)
    k = fn(_n3(b.shape), bc, pc, _ptr(b), _ptr(x), float(eps), int(max_iter), _ptr(hist))
    if k < 0:
        raise ValueError(f"oracle solver failed ({k})")
    return x, hist[:k + 1]


def pcg(b, bc=PERIODIC, pc=PC_STENCIL7, eps=1e-4, max_iter=1000, x0=None):
    """Textbook PCG: (x, eps history); len(history) - 1 iterations."""
    return _solve(lib().ryo_pcg, b, bc, pc, eps, max_iter, x0)


def ppcg(b, bc=PERIODIC, pc=PC_STENCIL7, eps=1e-4, max_iter=1000, x0=None):
    """Pipelined PCG (Ghysels & Vanroose Alg. 4): (x, eps history)."""
    return _solve(lib().ryo_ppcg, b, bc, pc, eps, max_iter, x0)


class PPCG:
    """Step-by-step PPCG on an explicit state (numpy arrays, x fastest)."""

    NAMES = ("x", "r", "u", "w", "z", "q", "s", "p")

    def __init__(self, b, bc=PERIODIC, pc=PC_STENCIL7, x0=None):
        self.b = _f64(b)
        self.shape = self.b.shape
        self.bc, self.pc = bc, pc
        self.v = {k: np.zeros(self.shape) for k in self.NAMES}
        self.st = PPCGState()
        self._bind()
        x0a = None if x0 is None else _f64(x0)
        lib().ryo_ppcg_init(_n3(self.shape), bc, pc, _ptr(self.b), None if x0a is None else _ptr(x0a),
                            C.byref(self.st))

    def _bind(self):
        for k in self.NAMES:
            setattr(self.st, k, self.v[k].ctypes.data_as(C.POINTER(C.c_double)))

    def set_state(self, vecs: dict, alpha_prev: float, gamma_prev: float, i: int):
        for k in self.NAMES:
            self.v[k][...] = vecs[k]
        self.st.alpha_prev, self.st.gamma_prev, self.st.i = alpha_prev, gamma_prev, i

    def dots(self):
        g, d = C.c_double(), C.c_double()
        lib().ryo_ppcg_dots(_n3(self.shape), C.byref(self.st), C.byref(g), C.byref(d))
        return g.value, d.value

    def step(self, gamma=None, delta=None):
        if gamma is None:
            gamma, delta = self.dots()
        lib().ryo_ppcg_step(_n3(self.shape), self.bc, self.pc, C.byref(self.st), gamma, delta)

    @property
    def i(self):
        return self.st.i

    @property
    def alpha_prev(self):
        return self.st.alpha_prev

    @property
    def gamma_prev(self):
        return self.st.gamma_prev
