"""Pins of the Poisson-solver oracle (oracle/poisson.c) to facts outside it.

The operator and the preconditioner are pinned by their closed-form
eigenpairs (Fourier modes on the periodic grid, sine modes under zero
Dirichlet) and by symmetry; the solvers by a dense LAPACK solve, an FFT
solve, SciPy's conjugate-gradient iterates, finite termination on a
two-eigenvalue right-hand side, monotone energy-norm error and the
iteration saving the paper reports for the preconditioner (Sec. 3.2).
"""
import numpy as np
import pytest
from scipy.sparse.linalg import LinearOperator, cg

from oracle import poisson as P


def grid(n, fn):
    """Array a[k, j, i] = fn(i, j, k) on an n = (n0, n1, n2) grid (x fastest)."""
    k, j, i = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    return fn(i.astype(float), j.astype(float), k.astype(float))


def smooth_rhs(n, seed, sigma=3.0):
    """Mean-free, smoothed Gaussian noise (the solver test workload's shape)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n[2], n[1], n[0]))
    f = np.fft.fftn(a)
    kz = np.fft.fftfreq(n[2])[:, None, None]
    ky = np.fft.fftfreq(n[1])[None, :, None]
    kx = np.fft.fftfreq(n[0])[None, None, :]
    f *= np.exp(-2 * (np.pi * sigma) ** 2 * (kx ** 2 + ky ** 2 + kz ** 2))
    b = np.fft.ifftn(f).real
    return b - b.mean()


# ------------------------------------------------------------ eigenpairs
@pytest.mark.parametrize("k", [(1, 2, 3), (0, 0, 1), (3, 1, 0), (4, 3, 5)])
def test_A_and_Minv_fourier_modes_periodic(k):
    n = (8, 6, 10)
    th = [2 * np.pi * k[d] / n[d] for d in range(3)]
    f = grid(n, lambda i, j, kk: np.cos(th[0] * i + th[1] * j + th[2] * kk + 0.3))
    lam = sum(2 - 2 * np.cos(t) for t in th)
    mu = 13 / 12 + sum(np.cos(t) for t in th) / 3
    np.testing.assert_allclose(P.apply_A(f, P.PERIODIC), lam * f, atol=1e-13)
    np.testing.assert_allclose(P.apply_Minv(f, P.PERIODIC), mu * f, atol=1e-13)
    np.testing.assert_array_equal(P.apply_Minv(f, P.PERIODIC, P.PC_NONE), f)


@pytest.mark.parametrize("k", [(1, 1, 1), (2, 3, 1), (5, 1, 4)])
def test_A_and_Minv_sine_modes_dirichlet(k):
    n = (7, 5, 6)
    th = [np.pi * k[d] / (n[d] + 1) for d in range(3)]
    f = grid(n, lambda i, j, kk: np.sin(th[0] * (i + 1)) * np.sin(th[1] * (j + 1)) * np.sin(th[2] * (kk + 1)))
    lam = sum(2 - 2 * np.cos(t) for t in th)
    mu = 13 / 12 + sum(np.cos(t) for t in th) / 3
    np.testing.assert_allclose(P.apply_A(f, P.DIRICHLET), lam * f, atol=1e-13)
    np.testing.assert_allclose(P.apply_Minv(f, P.DIRICHLET), mu * f, atol=1e-13)


@pytest.mark.parametrize("bc", [P.PERIODIC, P.DIRICHLET])
def test_operators_symmetric(bc):
    rng = np.random.default_rng(3)
    n = (5, 7, 3)
    x = rng.standard_normal((n[2], n[1], n[0]))
    y = rng.standard_normal((n[2], n[1], n[0]))
    for op in (lambda v: P.apply_A(v, bc), lambda v: P.apply_Minv(v, bc)):
        assert abs(np.vdot(op(x), y) - np.vdot(x, op(y))) < 1e-12 * np.abs(x).sum()


# ------------------------------------------------------------ solutions
def dense_laplacian_dirichlet(n):
    """The 7-point negative Laplacian as a dense matrix, by enumerating the
    face-neighbour pairs of the grid."""
    N = n[0] * n[1] * n[2]
    A = np.zeros((N, N))
    idx = lambda i, j, k: i + n[0] * (j + n[1] * k)
    for k in range(n[2]):
        for j in range(n[1]):
            for i in range(n[0]):
                c = idx(i, j, k)
                A[c, c] = 6.0
                for di, dj, dk in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
                    ii, jj, kk = i + di, j + dj, k + dk
                    if ii < n[0] and jj < n[1] and kk < n[2]:
                        A[c, idx(ii, jj, kk)] = A[idx(ii, jj, kk), c] = -1.0
    return A


@pytest.mark.parametrize("solver", [P.pcg, P.ppcg])
@pytest.mark.parametrize("pc", [P.PC_NONE, P.PC_STENCIL7])
def test_solution_matches_dense_solve_dirichlet(solver, pc):
    n = (4, 3, 5)
    rng = np.random.default_rng(11)
    b = rng.standard_normal((n[2], n[1], n[0]))
    xs = np.linalg.solve(dense_laplacian_dirichlet(n), b.ravel()).reshape(b.shape)
    x, hist = solver(b, P.DIRICHLET, pc, eps=1e-14, max_iter=200)
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-10 * np.abs(xs).max())
    assert hist[0] == 1.0


@pytest.mark.parametrize("solver", [P.pcg, P.ppcg])
def test_solution_matches_fft_solve_periodic(solver):
    n = (16, 12, 8)
    b = smooth_rhs(n, 5, sigma=1.0)
    bf = np.fft.fftn(b)
    lam = sum(2 - 2 * np.cos(2 * np.pi * np.fft.fftfreq(m))[s]
              for m, s in zip((n[2], n[1], n[0]), ((slice(None), None, None), (None, slice(None), None),
                                                   (None, None, slice(None)))))
    lam[0, 0, 0] = 1.0
    bf[0, 0, 0] = 0.0
    xs = np.fft.ifftn(bf / lam).real
    x, _ = solver(b, P.PERIODIC, P.PC_STENCIL7, eps=1e-13, max_iter=500)
    x = x - x.mean()
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-9 * np.abs(xs).max())


def test_ppcg_iterates_match_scipy_cg():
    """PPCG is PCG in exact arithmetic: its iterates follow SciPy's
    preconditioned CG (same x0 = 0, same operator and preconditioner)."""
    n = (10, 9, 8)
    b = smooth_rhs(n, 7, sigma=1.5)
    shp = b.shape
    N = b.size
    A = LinearOperator((N, N), matvec=lambda v: P.apply_A(v.reshape(shp), P.DIRICHLET).ravel(), dtype=float)
    M = LinearOperator((N, N), matvec=lambda v: P.apply_Minv(v.reshape(shp), P.DIRICHLET).ravel(), dtype=float)
    its = []
    cg(A, b.ravel(), M=M, rtol=1e-30, maxiter=12, callback=lambda xk: its.append(xk.copy()))
    st = P.PPCG(b, P.DIRICHLET, P.PC_STENCIL7)
    for k, xk in enumerate(its):
        st.step()
        np.testing.assert_allclose(st.v["x"].ravel(), xk, rtol=0, atol=1e-9 * np.abs(xk).max(),
                                   err_msg=f"iterate {k + 1}")


@pytest.mark.parametrize("pc", [P.PC_NONE, P.PC_STENCIL7])
def test_finite_termination_two_eigenvalues(pc):
    """A right-hand side in two eigenspaces of M^-1 A is solved exactly in
    two Krylov steps."""
    n = (8, 8, 8)
    t1, t2 = 2 * np.pi / 8, 2 * np.pi * 3 / 8
    b = grid(n, lambda i, j, k: np.cos(t1 * i + 0.2) + 0.5 * np.cos(t2 * j + t1 * k))
    for solver in (P.pcg, P.ppcg):
        x, hist = solver(b, P.PERIODIC, pc, eps=1e-12, max_iter=10)
        assert len(hist) - 1 == 2, hist
        np.testing.assert_allclose(P.apply_A(x, P.PERIODIC), b, atol=1e-12)


def test_energy_norm_error_decreases():
    n = (12, 12, 12)
    b = smooth_rhs(n, 9, sigma=1.0) + 0.1
    xs, _ = P.pcg(b, P.DIRICHLET, P.PC_STENCIL7, eps=1e-14, max_iter=500)
    st = P.PPCG(b, P.DIRICHLET, P.PC_STENCIL7)
    prev = np.inf
    for _ in range(20):
        e = st.v["x"] - xs
        en = float(np.vdot(e, P.apply_A(e, P.DIRICHLET)))
        assert en < prev
        prev = en
        st.step()


def test_pipelined_and_textbook_agree():
    n = (16, 16, 16)
    b = smooth_rhs(n, 13, sigma=2.0)
    _, h1 = P.pcg(b, P.PERIODIC, P.PC_STENCIL7, eps=1e-8, max_iter=300)
    _, h2 = P.ppcg(b, P.PERIODIC, P.PC_STENCIL7, eps=1e-8, max_iter=300)
    assert len(h1) == len(h2)
    np.testing.assert_allclose(h2[:15], h1[:15], rtol=1e-8)


def test_recursive_residual_tracks_true_residual():
    n = (12, 10, 8)
    b = smooth_rhs(n, 17, sigma=1.0)
    st = P.PPCG(b, P.PERIODIC, P.PC_STENCIL7)
    for _ in range(25):
        st.step()
    true_r = b - P.apply_A(st.v["x"], P.PERIODIC)
    assert np.abs(st.v["r"] - true_r).max() < 1e-10 * np.abs(b).max()
    np.testing.assert_allclose(st.v["u"], P.apply_Minv(st.v["r"], P.PERIODIC), atol=1e-10 * np.abs(b).max())


def test_preconditioner_halves_iterations():
    """The paper reports ~1.86x fewer iterations to eps = 1e-4 with the
    preconditioned pipelined solver (Sec. 3.2); the ratio is a property of
    the operator pair, close to 2 for any smooth right-hand side."""
    n = (32, 32, 32)
    b = smooth_rhs(n, 21, sigma=4.0)
    _, hcg = P.pcg(b, P.PERIODIC, P.PC_NONE, eps=1e-4, max_iter=2000)
    _, hpp = P.ppcg(b, P.PERIODIC, P.PC_STENCIL7, eps=1e-4, max_iter=2000)
    ratio = (len(hcg) - 1) / (len(hpp) - 1)
    assert 1.5 <= ratio <= 2.5, ratio


def test_zero_rhs_and_bad_arguments():
    b = np.zeros((4, 4, 4))
    x, hist = P.ppcg(b, P.PERIODIC, P.PC_STENCIL7)
    assert len(hist) == 1 and hist[0] == 0.0 and not x.any()
    with pytest.raises(ValueError):
        P.pcg(b, 7, P.PC_NONE)
