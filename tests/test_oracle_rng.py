"""Pins of the oracle's random inputs: Philox4x32-10, the open uniform, the
Box-Muller normals and the stratified start sampler (Algorithm "stratify",
assumption (A_nu) of the paper)."""
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import integrate, stats

import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _rocrand_reference(blocks):
    """Philox4x32-10 blocks from rocRAND's engine (an independent source)."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available to build the rocRAND reference")
    exe = os.path.join("/tmp", f"srmdp_philox_ref_{os.getpid()}")
    src = os.path.join(HERE, "helpers", "philox_rocrand_ref.cpp")
    subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950", src, "-o", exe],
                   check=True, capture_output=True, cwd="/tmp")
    try:
        inp = "\n".join(" ".join(str(v) for v in b) for b in blocks) + "\n"
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    finally:
        os.remove(exe)
    return np.array([[int(w) for w in line.split()] for line in out.strip().splitlines()],
                    dtype=np.uint64)


def test_philox_matches_rocrand_engine():
    rng = np.random.default_rng(12345)
    blocks = [[0, 0, 0, 0, 0, 0], [1, 0, 0, 0, 1, 0],
              [0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF]]
    blocks += rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64).tolist()
    ref = _rocrand_reference(blocks)
    mine = np.array([O.philox4x32_10(b[:4], b[4:]) for b in blocks], dtype=np.uint64)
    np.testing.assert_array_equal(mine, ref)


def test_uniform_is_open_and_exact():
    u = O.path_uniforms(seed=7, inst=3, i=5, k=11, m=2, n=4000)
    assert np.all(u > 0.0) and np.all(u < 1.0)
    # every value is (odd integer) * 2^-24: exactly representable in binary32
    scaled = u * 2.0**24
    assert np.all(scaled == np.round(scaled))
    assert np.all(np.round(scaled).astype(np.int64) % 2 == 1)
    assert np.all(u.astype(np.float32).astype(np.float64) == u)
    # the uniform is built from the top 23 bits of the Philox word
    w = O.philox4x32_10([0, 2, 11, 5 | (3 << 16)], [7, 0])
    expect = (2.0 * (w.astype(np.float64) // 512) + 1.0) * 2.0**-24
    np.testing.assert_array_equal(u[:4], expect)


def test_uniform_stream_counter_layout():
    # uniform n of simulation (i, k, m) is word n % 4 of block n / 4, counter
    # (block, m, k, i | inst << 16), key (seed low, seed high)
    seed = (5 << 32) | 9
    u = O.path_uniforms(seed, 2, 4, 77, 13, 12)
    for blk in range(3):
        w = O.philox4x32_10([blk, 13, 77, 4 | (2 << 16)], [9, 5])
        np.testing.assert_array_equal(u[4 * blk:4 * blk + 4],
                                      (2.0 * (w.astype(np.float64) // 512) + 1.0) * 2.0**-24)


def test_uniform_distribution_ks():
    u = np.concatenate([O.path_uniforms(1, 0, 0, k, 0, 64) for k in range(3000)])
    assert stats.kstest(u, "uniform").pvalue > 1e-4


def _prob(d=1, **kw):
    base = dict(d=d, N=10, lo=[-4.0] * d, hi=[4.0] * d, cells=[32] * d, M=8)
    base.update(kw)
    return O.Problem(**base)


def test_normals_moments_and_ks():
    P = _prob(d=1)
    n = np.concatenate([O.path_normals(P, 0, k, m, 40) for k in range(32) for m in range(60)])
    assert abs(n.mean()) < 5 / math.sqrt(n.size)
    assert abs(n.var() - 1.0) < 5 * math.sqrt(2.0 / n.size)
    assert stats.kstest(n, "norm").pvalue > 1e-4


def test_normals_are_box_muller_of_the_stream():
    """Normal l of path step s is number n = s Q + l of the path's normal
    sequence, Q = q when q divides 4 and 4 ceil(q/4) otherwise (a step starts
    on a Philox block of its own); number n is the cosine (even n) or sine (odd
    n) branch of Box-Muller on the uniforms 4 ceil(d/4) + 2 (n // 2) and + 1 of
    the same stream."""
    for d in (1, 2, 3, 4, 5, 8):
        P = _prob(d=d)
        steps = 3
        n = O.path_normals(P, 3, 5, 7, steps * d)
        Q = d if 4 % d == 0 else 4 * ((d + 3) // 4)
        b = 4 * ((d + 3) // 4)
        u = O.path_uniforms(P.seed, P.inst, 3, 5, 7, b + steps * Q + 2)
        for s in range(steps):
            for l in range(d):
                num = s * Q + l
                u1, u2 = u[b + 2 * (num // 2)], u[b + 2 * (num // 2) + 1]
                rho = math.sqrt(-2.0 * math.log(u1))
                ref = rho * (math.cos if num % 2 == 0 else math.sin)(2 * math.pi * u2)
                assert n[s * d + l] == pytest.approx(ref, rel=1e-14, abs=1e-15), (d, s, l)


def test_normals_uncorrelated_across_lags():
    P = _prob(d=1)
    n = np.stack([O.path_normals(P, 0, k, m, 16) for k in range(32) for m in range(100)])
    c = np.corrcoef(n.T)
    off = c[~np.eye(16, dtype=bool)]
    assert np.max(np.abs(off)) < 5 / math.sqrt(n.shape[0])


def test_streams_differ_across_step_cube_instance():
    a = O.path_uniforms(1, 0, 0, 0, 0, 8)
    for args in [(1, 0, 1, 0, 0), (1, 0, 0, 1, 0), (1, 0, 0, 0, 1), (1, 1, 0, 0, 0), (2, 0, 0, 0, 0)]:
        assert not np.array_equal(a, O.path_uniforms(*args, 8))


# ---------------------------------------------------------- start sampler --

def _logistic_cdf(x, mu=1.0):
    return 1.0 / (1.0 + np.exp(-mu * x))


def _truncated_mean(a, b, mu=1.0):
    # closed form: int x p(x) dx = x F(x) - log(1 + e^{mu x}) / mu
    def prim(x):
        return x * _logistic_cdf(x, mu) - np.log1p(np.exp(mu * x)) / mu
    return (prim(b) - prim(a)) / (_logistic_cdf(b, mu) - _logistic_cdf(a, mu))


def test_truncated_mean_closed_form_against_quadrature():
    for (a, b) in [(0.0, 0.25), (2.25, 3.0), (3.75, 4.0), (-4.0, -3.5)]:
        num = integrate.quad(lambda x: x * math.exp(-x) / (1 + math.exp(-x)) ** 2, a, b)[0]
        den = integrate.quad(lambda x: math.exp(-x) / (1 + math.exp(-x)) ** 2, a, b)[0]
        assert _truncated_mean(a, b) == pytest.approx(num / den, rel=1e-10)
    # printed values for mu = 1
    assert _truncated_mean(0.0, 0.25) == pytest.approx(0.1246755, abs=5e-7)
    assert _truncated_mean(2.25, 3.0) == pytest.approx(2.5849040, abs=5e-7)
    assert _truncated_mean(3.75, 4.0) == pytest.approx(3.8700090, abs=5e-7)


@pytest.mark.parametrize("cell,mu", [(16, 1.0), (21, 1.0), (31, 1.0), (2, 2.5), (29, 0.5)])
def test_start_sampler_in_cube_ks_and_mean(cell, mu):
    P = _prob(d=1, mu=mu)
    a = -4.0 + cell * 0.25
    b = a + 0.25
    x = np.array([O.start_point(P, 3, cell, m)[0] for m in range(4000)])
    assert np.all(x >= a) and np.all(x < b)
    cdf = lambda v: (_logistic_cdf(v, mu) - _logistic_cdf(a, mu)) / (
        _logistic_cdf(b, mu) - _logistic_cdf(a, mu))
    assert stats.kstest(x, cdf).pvalue > 1e-4
    var = integrate.quad(lambda v: (v - _truncated_mean(a, b, mu)) ** 2 * mu * math.exp(-mu * v) /
                         (1 + math.exp(-mu * v)) ** 2, a, b)[0] / (
        _logistic_cdf(b, mu) - _logistic_cdf(a, mu))
    assert abs(x.mean() - _truncated_mean(a, b, mu)) < 5 * math.sqrt(var / x.size)


def test_start_sampler_multidim_cube_order():
    # cube index: dimension 0 varies fastest
    P = O.Problem(d=3, N=4, lo=[-3, -2, -1], hi=[3, 2, 1], cells=[3, 4, 2], M=4)
    for k in [0, 1, 5, 13, 23]:
        c0, c1, c2 = k % 3, (k // 3) % 4, k // 12
        for m in range(20):
            x = O.start_point(P, 1, k, m)
            assert -3 + 2 * c0 <= x[0] < -3 + 2 * (c0 + 1)
            assert -2 + 1 * c1 <= x[1] < -2 + 1 * (c1 + 1)
            assert -1 + 1 * c2 <= x[2] < -1 + 1 * (c2 + 1)


def test_start_sampler_uses_the_first_uniforms():
    P = _prob(d=1)
    u = O.path_uniforms(P.seed, P.inst, 2, 20, 3, 1)[0]
    a, b = 1.0, 1.25
    Fa, Fb = _logistic_cdf(a), _logistic_cdf(b)
    expect = -math.log(1.0 / (Fa + u * (Fb - Fa)) - 1.0)
    assert O.start_point(P, 2, 20, 3)[0] == pytest.approx(expect, rel=1e-13)
