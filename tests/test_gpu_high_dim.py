"""The dimensions without the LDS kernel, d = 7, 9, 10 and 11..19 (the paper's
Tables LP0d11 and LP1d11 .. LP1d15_19): binary32 sweeps with the clouds in
global memory, per step against the FP64 oracle from the same rows (GPU tests,
through the C ABI)."""
import sys

import numpy as np
import pytest

import test_gpu_parity as TP
import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _logistic(d, cells, M, N, basis="LP1"):
    return dict(W.config("cfg2"), name=f"logistic d={d} K={int(np.prod(cells))} M={M} N={N} {basis} fp32", d=d,
                N=N, lo=[-3.0] * d, hi=[3.0] * d, cells=cells, M=M, basis=basis)


@pytest.mark.parametrize("d,cells,M,basis", [
    (7, [2] * 7, 40, "LP1"),
    (9, [2] * 5 + [1] * 4, 40, "LP1"),
    (10, [3] * 3 + [1] * 7, 32, "LP0"),
    (11, [2] * 6 + [1] * 5, 48, "LP1"),
    (13, [2] * 5 + [1] * 8, 40, "LP1"),
    (16, [2] * 8 + [1] * 8, 64, "LP1"),
    (12, [3] * 4 + [1] * 8, 32, "LP0"),
    (17, [2] * 6 + [1] * 11, 40, "LP1"),
    (18, [3] * 3 + [1] * 15, 32, "LP0"),
    (19, [2] * 7 + [1] * 12, 48, "LP1"),
])
def test_high_dimension_per_step_parity(d, cells, M, basis):
    """The logistic BSDE (look-up mode YZ) at d = 11, 13, 16 (LP1) and 12 (LP0),
    each step against the oracle's step from the same rows, at the FP32 bound."""
    cfg = _logistic(d, cells, M, N=3, basis=basis)
    err, excess, share = TP.fp32_step_parity(cfg, [2, 1, 0])
    assert err <= TP.TOL["fp32"]
    assert share < 0.1
    assert excess <= 0.0


def test_high_dimension_linear_driver_and_readouts():
    """d = 14, the cos terminal and the linear driver (look-up mode Y): per step
    against the oracle; then the read-outs of the oracle's own table in binary64
    (TABLE at sample points and ROOT from x0) against the oracle's."""
    import oracle as O
    from sides import oracle_problem, product_args
    import paper_2407_21085_amd as S
    torch = TP._torch()
    d = 14
    cfg = dict(W.config("cfg1"), name="cos d=14", d=d, N=3, lo=[-2.0] * d, hi=[2.0] * d, cells=[2] * 4 + [1] * 10,
               M=48, prec="fp32", r=0.1)
    err, excess, share = TP.fp32_step_parity(cfg, [2, 1, 0])
    assert err <= TP.TOL["fp32"]
    assert excess <= 0.0
    c64 = dict(cfg, prec="fp64")
    Po = oracle_problem(c64)
    orc, _ = O.solve(Po)
    P, G, Opt = product_args(c64)
    table = torch.from_numpy(orc).cuda()
    x0 = [0.1] * d
    _say("[gpu] d = 14 read-outs of the oracle's table")
    y0, z0 = S.root(P, G, Opt, table, x0, 20000)
    yo, zo = O.root(Po, orc, x0, 20000)
    assert y0 == pytest.approx(yo, rel=1e-9)
    np.testing.assert_allclose(z0, zo, rtol=1e-8, atol=1e-10)
    pts = np.random.default_rng(3).uniform(-2.5, 2.5, (257, d))
    y, z = S.evaluate(P, G, Opt.basis, Opt.prec, table, 1, torch.from_numpy(pts).cuda())
    ye, ze = O.evaluate(Po, orc, 1, pts)
    np.testing.assert_allclose(y.cpu().numpy(), ye, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(z.cpu().numpy(), ze, rtol=1e-12, atol=1e-14)
