"""Pins of the oracle's least-squares steps (Definition "Ordinary linear
least-squares regression", Section "Explicit solutions to OLS") against
routes that share nothing with it: numpy's lstsq, a Householder QR written
here (the paper's LP1 route), the LP0 closed form (the empirical mean) and
exact interpolation when M = d + 1."""
import math

import numpy as np
import pytest

import oracle as O


def householder_qr_solve(A, S):
    """Least squares by Householder reflections, then R alpha = Q^T S."""
    A = np.array(A, dtype=np.float64)
    b = np.array(S, dtype=np.float64).reshape(A.shape[0], -1)
    m, n = A.shape
    for c in range(n):
        x = A[c:, c]
        v = x.copy()
        v[0] += math.copysign(np.linalg.norm(x), x[0])
        v /= np.linalg.norm(v)
        A[c:, :] -= 2.0 * np.outer(v, v @ A[c:, :])
        b[c:, :] -= 2.0 * np.outer(v, v @ b[c:, :])
    R = np.triu(A[:n, :n])
    out = np.zeros((n, b.shape[1]))
    for r in range(n - 1, -1, -1):
        out[r] = (b[r] - R[r, r + 1:] @ out[r + 1:]) / R[r, r]
    return out


def _centred_basis(P, k, X):
    """(1, xi_1..xi_d) with xi = 2 (x - centre) / h; the cube index has
    dimension 0 fastest."""
    cells = np.asarray(P.cells)
    lo = np.asarray(P.lo, dtype=float)
    h = (np.asarray(P.hi, dtype=float) - lo) / cells
    idx, kk = [], k
    for c in cells:
        idx.append(kk % c)
        kk //= c
    centre = lo + (np.asarray(idx) + 0.5) * h
    return np.hstack([np.ones((X.shape[0], 1)), 2.0 * (X - centre) / h])


def _fits_by_lstsq(P, tab, i, k, solver):
    """z then y regressions of one stratum, recomputed from its cloud with a
    least-squares route of the test's own, for the linear driver
    f = -r y + kappa sum(z)."""
    Xi, dW, Sp, y1, cvi = O.cloud(P, tab, i, k)
    A = _centred_basis(P, k, Xi) if P.basis == O.LP1 else np.ones((P.M, 1))
    Rz = Sp[:, None] * dW / P.dt
    bz = solver(A, Rz)                       # (nb, q)
    zfit = A @ bz                            # (M, q)
    SY = Sp + (-P.r * y1 + P.kappa * zfit.sum(axis=1)) * P.dt - cvi
    by = solver(A, SY[:, None])[:, 0]
    return by, bz.T, A, SY, Rz


def _lstsq(A, B):
    return np.linalg.lstsq(A, B, rcond=None)[0]


@pytest.mark.parametrize("solver", [_lstsq, householder_qr_solve], ids=["lstsq", "householder"])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_lp1_fit_matches_bruteforce_least_squares(solver, d):
    P = O.Problem(d=d, N=3, lo=[-1.5] * d, hi=[1.5] * d, cells=[2] * d, M=8, r=0.7, kappa=0.4,
                  seed=11)
    tab, sing = O.solve(P)
    assert sing == 0
    for i in range(P.N):
        for k in range(P.K):
            by, bz, *_ = _fits_by_lstsq(P, tab, i, k, solver)
            np.testing.assert_allclose(tab[i, k, 0], by, rtol=1e-9, atol=1e-11)
            np.testing.assert_allclose(tab[i, k, 1:], bz, rtol=1e-9, atol=1e-11)


def test_lp0_fit_is_the_empirical_mean():
    P = O.Problem(d=2, N=4, lo=[-2, -2], hi=[2, 2], cells=[3, 3], M=50, r=0.3, kappa=-0.2,
                  basis=O.LP0, seed=5)
    tab, _ = O.solve(P)
    for i in range(P.N):
        for k in range(P.K):
            Xi, dW, Sp, y1, cvi = O.cloud(P, tab, i, k)
            zbar = (Sp[:, None] * dW / P.dt).mean(axis=0)
            SY = Sp + (-P.r * y1 + P.kappa * zbar.sum()) * P.dt
            assert tab[i, k, 0, 0] == pytest.approx(SY.mean(), rel=1e-13, abs=1e-15)
            np.testing.assert_allclose(tab[i, k, 1:, 0], zbar, rtol=1e-13, atol=1e-15)


def test_lp1_residuals_orthogonal_to_basis():
    P = O.Problem(d=3, N=3, lo=[-2] * 3, hi=[2] * 3, cells=[2] * 3, M=40, r=0.2, kappa=0.3,
                  seed=2)
    tab, _ = O.solve(P)
    for k in range(P.K):
        by, bz, A, SY, Rz = _fits_by_lstsq(P, tab, 0, k, _lstsq)
        res_y = SY - A @ tab[0, k, 0]
        res_z = Rz - A @ tab[0, k, 1:].T
        scale = np.abs(A).sum() * (np.abs(SY).max() + np.abs(Rz).max())
        assert np.max(np.abs(A.T @ res_y)) < 1e-11 * scale
        assert np.max(np.abs(A.T @ res_z)) < 1e-11 * scale
        assert abs(res_y.sum()) < 1e-11 * scale   # the constant is in the basis


def test_lp1_interpolates_when_M_equals_dimension():
    d = 2
    P = O.Problem(d=d, N=2, lo=[-1, -1], hi=[1, 1], cells=[2, 2], M=d + 1, r=0.5, seed=9)
    tab, _ = O.solve(P)
    for k in range(P.K):
        by, bz, A, SY, Rz = _fits_by_lstsq(P, tab, 0, k, _lstsq)
        np.testing.assert_allclose(A @ tab[0, k, 0], SY, rtol=1e-9, atol=1e-10)
        np.testing.assert_allclose(A @ tab[0, k, 1:].T, Rz, rtol=1e-9, atol=1e-10)


def test_single_step_hand_algebra():
    # N = 1: z_0 = OLS(g(X_1) dW_0 / dt), y_0 = OLS(g(X_1) + f(t_0, X_0, g(X_1), z_0(X_0)) dt)
    P = O.Problem(d=1, N=1, lo=[-2], hi=[2], cells=[4], M=30, r=1.3, kappa=0.8, seed=4)
    tab, _ = O.solve(P)
    for k in range(P.K):
        Xi, dW, Sp, y1, cvi = O.cloud(P, tab, 0, k)
        X1 = Xi[:, 0] + dW[:, 0]
        np.testing.assert_allclose(Sp, np.cos(X1), rtol=1e-13)
        np.testing.assert_allclose(y1, np.cos(X1), rtol=1e-13)
        A = _centred_basis(P, k, Xi)
        bz = _lstsq(A, np.cos(X1) * dW[:, 0] / P.dt)
        SY = np.cos(X1) + (-P.r * np.cos(X1) + P.kappa * (A @ bz)) * P.dt
        by = _lstsq(A, SY)
        np.testing.assert_allclose(tab[0, k, 1], bz, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(tab[0, k, 0], by, rtol=1e-10, atol=1e-12)


def test_threads_do_not_change_results():
    P = O.Problem(d=2, N=5, lo=[-2, -2], hi=[2, 2], cells=[4, 4], M=20, r=0.1, seed=3)
    t1, _ = O.solve(P, threads=1)
    t8, _ = O.solve(P, threads=8)
    np.testing.assert_array_equal(t1, t8)


def test_partial_sweep_resumes_exactly():
    P = O.Problem(d=1, N=8, lo=[-3], hi=[3], cells=[12], M=32, r=0.2, seed=3)
    full, _ = O.solve(P)
    part, _ = O.solve(P, i_hi=7, i_lo=4)
    part, _ = O.solve(P, table=part, i_hi=3, i_lo=0)
    np.testing.assert_array_equal(full, part)


def test_truncation_applies_at_evaluation():
    P = O.Problem(d=1, N=4, lo=[-3], hi=[3], cells=[12], M=64, r=0.0, seed=3)
    tab, _ = O.solve(P)
    x = np.linspace(-5, 5, 101)
    y, z = O.evaluate(P, tab, 1, x)
    P2 = O.Problem(d=1, N=4, lo=[-3], hi=[3], cells=[12], M=64, r=0.0, seed=3, clamp_y=0.3,
                   clamp_z=0.1)
    y2, z2 = O.evaluate(P2, tab, 1, x)
    np.testing.assert_array_equal(y2, np.clip(y, -0.3, 0.3))
    np.testing.assert_array_equal(z2, np.clip(z, -0.1, 0.1))


def test_evaluation_outside_domain_uses_boundary_cell_affine_fit():
    P = O.Problem(d=1, N=2, lo=[-1], hi=[1], cells=[4], M=64, seed=8)
    tab, _ = O.solve(P)
    xs = np.array([-3.0, -1.0, 0.0, 0.99, 2.5])
    y, _ = O.evaluate(P, tab, 0, xs)
    # cell 0 covers [-1, -0.5): centre -0.75, h = 0.5; cell 3 covers [0.5, 1)
    e0 = tab[0, 0, 0, 0] + tab[0, 0, 0, 1] * 2 * (-3.0 + 0.75) / 0.5
    e3 = tab[0, 3, 0, 0] + tab[0, 3, 0, 1] * 2 * (2.5 - 0.75) / 0.5
    assert y[0] == pytest.approx(e0, rel=1e-13)
    assert y[4] == pytest.approx(e3, rel=1e-13)
    # half-open cells: x = 0 belongs to the cell [0, 0.5)
    assert y[2] == pytest.approx(tab[0, 2, 0, 0] + tab[0, 2, 0, 1] * 2 * (0.0 - 0.25) / 0.5,
                                 rel=1e-13)


def test_invalid_problems_are_rejected():
    with pytest.raises(ValueError):
        O.solve(O.Problem(d=2, N=3, lo=[-1, -1], hi=[1, 1], cells=[2, 2], M=2))  # M < d+1
    with pytest.raises(ValueError):
        O.solve(O.Problem(d=1, N=3, lo=[1], hi=[-1], cells=[2], M=8))           # lo >= hi
    with pytest.raises(ValueError):
        O.solve(O.Problem(d=1, N=3, lo=[-1], hi=[1], cells=[0], M=8))           # no cells
