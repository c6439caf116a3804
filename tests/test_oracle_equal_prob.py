"""Pins of the oracle's equal-probability strata, the second example of
hypercubes under assumption (A_Strat): per dimension the C cells are cut at
the logistic quantiles F^{-1}(c / C), so that every cube has nu-probability
1/K under the law nu of assumption (A_nu) and the cubes cover R^d (the two
outer cells of each dimension are unbounded).

* the sampler draws nu_k: the probability coordinate C F(x_l) - c of every
  start point is uniform on [0, 1) (Kolmogorov-Smirnov), independently drawn
  points of the unrestricted law nu fall in each cube with frequency 1/K;
* the oracle's look-up (through the TABLE read-out with a table whose value
  in cube k is k) puts every start point of stratum k back in cube k;
* the fits tend to the nu_k-weighted projection of the discrete closed form
  of the cos family, computed by Gauss-Legendre quadrature in the probability
  coordinate (which turns the unbounded cells into [0, 1));
* with the driver coupled through y and z the read-out stays within the Monte
  Carlo band of the closed form, as for the equal-size grid.
"""
import math

import numpy as np
import pytest
from scipy import stats

import oracle as O
import test_oracle_closed_form as CF


def _prob(cells, mu=1.0, **kw):
    d = len(cells)
    kw.setdefault("N", 3)
    kw.setdefault("M", 64)
    return O.Problem(d=d, lo=None, hi=None, cells=cells, mu=mu,
                     grid_kind=O.GRID_EQUAL_PROB, **kw)


def _cdf(x, mu):
    return 1.0 / (1.0 + np.exp(-mu * np.asarray(x, float)))


def _cube_cells(cells, k):
    out = []
    for c in cells:
        out.append(k % c)
        k //= c
    return out


@pytest.mark.parametrize("mu,cells", [(1.3, [5, 3]), (0.6, [1, 7])])
def test_equal_probability_sampler_law(mu, cells):
    P = _prob(cells, mu)
    for k in sorted({0, P.K - 1, P.K // 2, 1}):
        cc = _cube_cells(cells, k)
        x = np.array([O.start_point(P, 1, k, m) for m in range(3000)])
        for l, n in enumerate(cells):
            t = n * _cdf(x[:, l], mu) - cc[l]
            assert np.all(t >= 0.0) and np.all(t < 1.0), (k, l)
            assert stats.kstest(t, "uniform").pvalue > 1e-4, (k, l)


@pytest.mark.parametrize("mu,cells", [(0.7, [4, 6]), (2.0, [3, 1, 2])])
def test_equal_probability_lookup_matches_strata(mu, cells):
    """Cube k's constant in a LP0 table is k: the read-out at a point names
    the cube the oracle's look-up puts it in."""
    P = _prob(cells, mu, basis=O.LP0)
    tab = np.zeros(P.table_shape())
    tab[:, :, 0, 0] = np.arange(P.K)[None, :]
    for k in range(P.K):
        x = np.array([O.start_point(P, 0, k, m) for m in range(40)])
        y, _ = O.evaluate(P, tab, 0, x)
        assert np.all(y == k), k
    # points of the unrestricted law nu (numpy's logistic generator): each
    # cube has probability 1/K
    rng = np.random.default_rng(11)
    n = 60000
    x = rng.logistic(0.0, 1.0 / mu, size=(n, len(cells)))
    y, _ = O.evaluate(P, tab, 0, x)
    counts = np.bincount(y.astype(np.int64), minlength=P.K)
    assert counts.size == P.K
    assert stats.chisquare(counts).pvalue > 1e-4


def _nu_proj_prob(fun, cells, cc, mu, npts=64):
    """nu_k-weighted L2 projection of fun on span{1, mu (x_l - m_l)} over the
    equal-probability cube with cell indices cc, m_l the cell's nu-median.
    Under nu_k the probability coordinates u_l = C_l F(x_l) - c_l are
    independent uniforms on [0, 1): quadrature in u, x = F^{-1}((c + u) / C)."""
    d = len(cells)
    us, ws = np.polynomial.legendre.leggauss(npts)
    us, ws = 0.5 * (us + 1.0), 0.5 * ws
    grids, med = [], []
    for l in range(d):
        p = (cc[l] + us) / cells[l]
        grids.append(np.log(p / (1.0 - p)) / mu)
        pm = (cc[l] + 0.5) / cells[l]
        med.append(math.log(pm / (1.0 - pm)) / mu)
    mesh = np.meshgrid(*grids, indexing="ij")
    wm = np.meshgrid(*([ws] * d), indexing="ij")
    W = np.prod(np.stack([w.ravel() for w in wm]), axis=0)
    X = np.stack([m.ravel() for m in mesh], axis=1)
    A = np.hstack([np.ones((X.shape[0], 1)), mu * (X - np.asarray(med))])
    G = (A * W[:, None]).T @ A
    return np.linalg.solve(G, (A * W[:, None]).T @ fun(X)), np.asarray(med)


@pytest.mark.parametrize("d,cells,N,M", [(1, [8], 3, 20000), (2, [4, 3], 2, 12000)])
def test_equal_probability_fits_match_projection(d, cells, N, M):
    """f = 0, g = cos(sum x): each LP1 coefficient, unbounded cells included,
    within 5 standard errors of the projection of the discrete closed form."""
    mu = 0.8
    P = _prob(cells, mu, N=N, M=M, seed=4)
    tab, sing = O.solve(P)
    assert sing == 0
    yex, zex = CF._cos_exact(P)
    worst = 0.0
    for i in range(N):
        for k in range(P.K):
            cc = _cube_cells(cells, k)
            Xi, dW, Sp, y1, cvi = O.cloud(P, tab, i, k)
            py, med = _nu_proj_prob(yex(i), cells, cc, mu)
            A = np.hstack([np.ones((M, 1)), mu * (Xi - med)])
            worst = max(worst, np.max(np.abs(tab[i, k, 0] - py) / CF._sandwich_se(A, Sp)))
            pz, _ = _nu_proj_prob(zex(i), cells, cc, mu)
            for l in range(P.q):
                se_z = CF._sandwich_se(A, Sp * dW[:, l] / P.dt)
                worst = max(worst, np.max(np.abs(tab[i, k, 1 + l] - pz) / se_z))
    assert worst < 5.0, worst


def test_equal_probability_coupled_driver_matches_discrete_closed_form():
    """r = 2, kappa = 1 on 24 equal-probability cells of R (mu = 1, so the
    inner cells span about [-3.1, 3.1]): the read-outs inside [-1.5, 1.5]
    stay within the band of the equal-size case."""
    P = _prob([24], 1.0, N=4, M=40000, r=2.0, kappa=1.0, seed=5)
    tab, _ = O.solve(P)
    yex, zex = CF._cos_exact(P)
    xs = np.linspace(-1.5, 1.5, 61)[:, None]
    for i in range(P.N):
        y, z = O.evaluate(P, tab, i, xs)
        assert np.max(np.abs(y - yex(i)(xs))) < 0.025
        assert np.max(np.abs(z[:, 0] - zex(i)(xs))) < 0.06
        assert abs(np.mean(y - yex(i)(xs))) < 0.004


def test_truncation_keeps_unbounded_strata_stable():
    """With two cells per dimension every cube is unbounded.  Its few far
    samples steer the LP1 slopes, and without truncation the logistic BSDE's
    fits grow over the 50 backward steps (d = 8, K = 256, M = 64: coefficients
    near 1e29 at step 0 for this seed); truncating y at C_y = 1, which bounds
    the solution, as the estimator of eq. (TL) does, keeps every coefficient of
    moderate size and y(0, 0) near its value 1/2."""
    kw = dict(N=50, M=64, driver=O.DRV_LOGISTIC, terminal=O.G_LOGISTIC, seed=1)
    tab, _ = O.solve(_prob([2] * 8, 1.0, **kw))
    assert np.nanmax(np.abs(tab[0])) > 1e6
    tab1, _ = O.solve(_prob([2] * 8, 1.0, clamp_y=1.0, **kw))
    assert np.all(np.isfinite(tab1)) and np.max(np.abs(tab1)) < 100.0
    y0, _ = O.root(_prob([2] * 8, 1.0, clamp_y=1.0, **kw), tab1, [0.0] * 8, 100000)
    assert abs(y0 - 0.5) < 0.05, y0
