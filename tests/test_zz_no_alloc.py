"""ry_cfl_dt_noalloc, the allocation-free CFL time step over a level held in
the caller's device memory, against ry_cfl_dt of a context holding the same
state: the same dt bit for bit on two calls in a row (the second with a
smaller input), leaf masks honoured, a latched numeric fault reported and
cleared for the next call, sizes beyond the scratch array rejected."""
from __future__ import annotations

import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ry():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2411_14631_amd import ry as mod
    mod.lib()
    return mod


def noalloc(ry):
    f = ry.lib().ry_cfl_dt_noalloc
    f.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double,
                  C.c_double, C.POINTER(C.c_double), C.c_void_p]
    f.restype = C.c_int32
    return f


def call(f, prob, Ud, n_oct, refined_d, plane=None):
    import torch
    dx = prob.boxlen / prob.nbase[0]
    dt = C.c_double(-1.0)
    torch.cuda.synchronize()
    rc = f(Ud.data_ptr(), 8 * n_oct if plane is None else plane, n_oct, refined_d.data_ptr(), prob.gamma, prob.cfl,
           dx, prob.rho_floor, prob.p_floor, C.byref(dt), None)
    return rc, dt.value


def test_noalloc_cfl_equals_context_cfl(ry):
    import torch
    f = noalloc(ry)
    for n in (32, 16):                       # the second call on a smaller input
        prob = W.random_smooth(n, seed=40 + n, mach=1.3)
        h = ry.Hydro(prob)
        h.advance(2)
        dt_ref = h.cfl_dt()
        U = h.download(prob.level_min)
        n_oct = U.shape[1] // 8
        Ud = torch.tensor(U, device="cuda")
        refd = torch.zeros(n_oct, dtype=torch.uint8, device="cuda")
        rc, dt = call(f, prob, Ud, n_oct, refd)
        assert rc == ry.RY_OK
        assert dt == dt_ref, (n, dt, dt_ref)
        # cells marked refined are left out: give them a far larger signal
        # speed, the time step stays that of the leaf cells
        V = U.copy()
        V[1, 3::64] *= 50.0
        V[4, 3::64] += 0.5 * V[1, 3::64] ** 2 / V[0, 3::64]
        mask = np.zeros(n_oct, np.uint8)
        mask[::8] = 1 << 3
        rc, dt2 = call(f, prob, torch.tensor(V, device="cuda"), n_oct, torch.tensor(mask, device="cuda"))
        assert rc == ry.RY_OK and dt2 == dt_ref
        rc, dt3 = call(f, prob, torch.tensor(V, device="cuda"), n_oct, refd)
        assert rc == ry.RY_OK and dt3 < 0.5 * dt_ref
        h.close()


def test_noalloc_cfl_fault_and_limits(ry):
    import torch
    f = noalloc(ry)
    prob = W.random_smooth(16, seed=5)
    U = prob.base_flat().copy()
    n_oct = U.shape[1] // 8
    refd = torch.zeros(n_oct, dtype=torch.uint8, device="cuda")
    bad = U.copy()
    bad[0, 17] = np.nan
    rc, _ = call(f, prob, torch.tensor(bad, device="cuda"), n_oct, refd)
    assert rc == ry.RY_ENUMERIC
    rc, dt = call(f, prob, torch.tensor(U, device="cuda"), n_oct, refd)   # the fault word was cleared
    assert rc == ry.RY_OK and np.isfinite(dt) and dt > 0
    Ud = torch.tensor(U, device="cuda")
    # beyond the scratch array (2M octs) or an inconsistent plane: refused
    # before any launch
    assert call(f, prob, Ud, (1 << 21) + 1, refd, plane=8 * ((1 << 21) + 1))[0] == ry.RY_EINVAL
    assert call(f, prob, Ud, n_oct, refd, plane=8 * n_oct - 1)[0] == ry.RY_EINVAL
    dt = C.c_double()
    assert f(None, 8 * n_oct, n_oct, refd.data_ptr(), 1.4, 0.8, 0.1, 1e-10, 1e-10, C.byref(dt), None) == ry.RY_EINVAL
