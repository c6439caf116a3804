"""Pins of the oracle with a problem's own coefficients (CPU only).

1. Plumbing: a C plugin that restates a built-in family (drift b + diag(b_lin)
   x, diffusion Sigma + diag(sigma_lin) x with a non-symmetric Sigma, the
   logistic or linear driver, the logistic or cos terminal) gives the
   built-in path's table bit for bit.  A transposed Sigma, a wrong time or a
   swapped argument would not.

2. Time dependence, through a discrete closed form.  With
   b(t, x) = (a0 + a1 t) 1, sigma = s I, f(t, x, y, z) = h(t) cos(x_1),
   h(t) = h0 + h1 t, g(x) = cos(sum x), the Euler chain is Gaussian:
   from X_i = x, sum X_j = sum x + d sum_{m=i}^{j-1} c_m dt + s sqrt(d) N(0, (j-i) dt),
   c_m = a0 + a1 t_m, t_m = m dt.  The MDP identity eq. (MDP:intro) with f
   free of y and z gives
     y_i(x) = e^{-s^2 d (N-i) dt / 2} cos(u + d C_{i,N})
              + sum_{j=i}^{N-1} h(t_j) dt e^{-s^2 (j-i) dt / 2} cos(x_1 + C_{i,j}),
     z_{i,l}(x) = -s e^{-s^2 d (N-i) dt / 2} sin(u + d C_{i,N})
              - [l = 1] s sum_{j=i+1}^{N-1} h(t_j) dt e^{-s^2 (j-i) dt / 2} sin(x_1 + C_{i,j}),
   u = sum x, C_{i,j} = sum_{m=i}^{j-1} c_m dt (Gaussian integration by parts
   in dW_i for z).  Every fitted coefficient must lie within 5 standard
   errors of the nu_k projection of these functions on the local space.
"""
import math

import numpy as np
import pytest

import oracle as O
from test_oracle_closed_form import _cube_bounds, _nu_proj, _sandwich_se

BUILTIN_PLUGIN = r"""
#include <math.h>
/* p: b[D], b_lin[D], Sigma[D*D] (row-major), sigma_lin[D], T, r, kappa, logistic driver flag,
 * logistic terminal flag */
#define D MODEL_D
void model_b(double t, const double *x, const double *p, double *out)
{
    (void)t;
    for (int l = 0; l < D; ++l) out[l] = p[l] + p[D + l] * x[l];
}
void model_sigma_dw(double t, const double *x, const double *dw, const double *p, double *out)
{
    (void)t;
    const double *S = p + 2 * D, *sl = p + 2 * D + D * D;
    for (int l = 0; l < D; ++l) {
        double acc = 0.0;
        for (int c = 0; c < D; ++c) acc += S[l * D + c] * dw[c];
        acc += sl[l] * x[l] * dw[l];
        out[l] = acc;
    }
}
double model_f(double t, const double *x, double y, const double *z, const double *p)
{
    (void)t;
    (void)x;
    const double *q = p + 3 * D + D * D;
    double sz = 0.0;
    for (int l = 0; l < D; ++l) sz += z[l];
    if (q[3] != 0.0) return sz * (y - (2.0 + D) / (2.0 * D));
    return -q[1] * y + q[2] * sz;
}
double model_g(const double *x, const double *p)
{
    const double *q = p + 3 * D + D * D;
    double s = 0.0;
    for (int l = 0; l < D; ++l) s += x[l];
    if (q[4] != 0.0) {
        double w = exp(q[0] + s);
        return w / (1.0 + w);
    }
    return cos(s);
}
"""

TIME_PLUGIN = r"""
#include <math.h>
/* p: a0, a1, s, h0, h1 */
#define D MODEL_D
void model_b(double t, const double *x, const double *p, double *out)
{
    (void)x;
    for (int l = 0; l < D; ++l) out[l] = p[0] + p[1] * t;
}
void model_sigma_dw(double t, const double *x, const double *dw, const double *p, double *out)
{
    (void)t;
    (void)x;
    for (int l = 0; l < D; ++l) out[l] = p[2] * dw[l];
}
double model_f(double t, const double *x, double y, const double *z, const double *p)
{
    (void)y;
    (void)z;
    return (p[3] + p[4] * t) * cos(x[0]);
}
double model_g(const double *x, const double *p)
{
    (void)p;
    double s = 0.0;
    for (int l = 0; l < D; ++l) s += x[l];
    return cos(s);
}
"""


def builtin_params(d, b, b_lin, Sigma, sigma_lin, T, r, kappa, logistic_driver, logistic_terminal):
    return (list(b) + list(b_lin) + list(np.asarray(Sigma, float).ravel()) + list(sigma_lin)
            + [T, r, kappa, float(logistic_driver), float(logistic_terminal)])


BUILTIN_CASES = [
    ("logistic d=3 ornstein-uhlenbeck full sigma", 3, dict(driver=O.DRV_LOGISTIC, terminal=O.G_LOGISTIC),
     dict(b=[0.1, -0.2, 0.05], b_lin=[-0.5, 0.2, 0.0],
          sigma=[0.9, 0.1, -0.05, 0.0, 1.1, 0.2, 0.15, -0.1, 0.8], sigma_lin=[0.3, 0.0, -0.2])),
    ("linear kappa d=2 cos", 2, dict(driver=O.DRV_LINEAR, terminal=O.G_COS_SUM, r=0.3, kappa=0.4),
     dict(b=[0.2, -0.1], b_lin=[0.0, -0.7], sigma=[1.0, 0.3, -0.2, 0.7], sigma_lin=[0.0, 0.4])),
]


@pytest.mark.parametrize("name,d,drv,coef", BUILTIN_CASES, ids=[c[0] for c in BUILTIN_CASES])
def test_plugin_restating_a_builtin_family_is_bit_identical(name, d, drv, coef):
    grid = dict(d=d, N=4, lo=[-2.0] * d, hi=[2.0] * d, cells=[3] * d, M=40, seed=5, T=1.0)
    ref, _ = O.solve(O.Problem(**grid, **drv, **coef))
    params = builtin_params(d, coef["b"], coef["b_lin"], np.reshape(coef["sigma"], (d, d)), coef["sigma_lin"],
                            1.0, drv.get("r", 0.0), drv.get("kappa", 0.0), drv["driver"] == O.DRV_LOGISTIC,
                            drv["terminal"] == O.G_LOGISTIC)
    model = O.Model(BUILTIN_PLUGIN, params)
    got, _ = O.solve(O.Problem(**grid, model=model))
    np.testing.assert_array_equal(got, ref)
    # the driver and terminal the oracle calls are the plugin's
    Pm = O.Problem(**grid, model=model)
    Pb = O.Problem(**grid, **drv, **coef)
    x, z = np.linspace(-1, 1, d), np.linspace(0.3, -0.2, d)
    assert O.driver(Pm, 0.2, x, 0.4, z) == O.driver(Pb, 0.2, x, 0.4, z)
    assert O.terminal(Pm, x) == O.terminal(Pb, x)


def time_model_exact(P, a0, a1, s, h0, h1):
    d, dt, N = P.d, P.dt, P.N
    c = [a0 + a1 * m * dt for m in range(N)]

    def C(i, j):
        return sum(c[m] for m in range(i, j)) * dt

    def h(t):
        return h0 + h1 * t

    def y(i):
        def f(X):
            u = X.sum(axis=1)
            v = math.exp(-s * s * d * (N - i) * dt / 2) * np.cos(u + d * C(i, N))
            for j in range(i, N):
                v = v + h(j * dt) * dt * math.exp(-s * s * (j - i) * dt / 2) * np.cos(X[:, 0] + C(i, j))
            return v
        return f

    def z(i, l):
        def f(X):
            u = X.sum(axis=1)
            v = -s * math.exp(-s * s * d * (N - i) * dt / 2) * np.sin(u + d * C(i, N))
            if l == 0:
                for j in range(i + 1, N):
                    v = v - s * h(j * dt) * dt * math.exp(-s * s * (j - i) * dt / 2) * np.sin(X[:, 0] + C(i, j))
            return v
        return f
    return y, z


@pytest.mark.parametrize("d,cells,N,M", [(1, [16], 4, 20000), (2, [4, 4], 3, 12000)])
def test_time_dependent_model_fits_match_projection_of_closed_form(d, cells, N, M):
    a0, a1, s, h0, h1 = 0.3, -0.8, 0.7, 0.4, 1.5
    model = O.Model(TIME_PLUGIN, [a0, a1, s, h0, h1])
    P = O.Problem(d=d, N=N, lo=[-2.0] * d, hi=[2.0] * d, cells=cells, M=M, seed=9, model=model)
    tab, sing = O.solve(P)
    assert sing == 0
    yex, zex = time_model_exact(P, a0, a1, s, h0, h1)
    worst = 0.0
    for i in range(N):
        for k in range(P.K):
            a, b = _cube_bounds(P, k)
            Xi, dW, Sp, y1, cvi = O.cloud(P, tab, i, k)
            cc, hh = 0.5 * (a + b), b - a
            A = np.hstack([np.ones((M, 1)), 2 * (Xi - cc) / hh])
            SY = Sp + (h0 + h1 * i * P.dt) * np.cos(Xi[:, 0]) * P.dt
            se_y = _sandwich_se(A, SY)
            worst = max(worst, np.max(np.abs(tab[i, k, 0] - _nu_proj(yex(i), a, b)) / se_y))
            for l in range(P.q):
                se_z = _sandwich_se(A, Sp * dW[:, l] / P.dt)
                worst = max(worst, np.max(np.abs(tab[i, k, 1 + l] - _nu_proj(zex(i, l), a, b)) / se_z))
    assert worst < 5.0, worst
