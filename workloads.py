"""Workload definitions shared by the tests, the smoke check and the benchmark.

Inputs only: problem data, grids, sizes and seeds of the synthetic workloads,
plus the seeded generator of the ragged batch.  Nothing here computes any part
of the method; both the HIP library's binding and the oracle receive these
plain values.

All workloads are the analytic BSDEs of the paper (no dataset is involved):
  * "cos" family: X = x0 + W, f = -r y (+ kappa sum z), g = cos(sum x);
  * "logistic": the benchmark of the paper's Section 5.1, f = (sum z)(y - (2+q)/(2q)),
    g = omega(T,x)/(1+omega(T,x)), omega(t,x) = exp(t + sum x).
"""
from __future__ import annotations

import copy
from typing import Dict, List

import numpy as np

# cfg1: d = q = 1, cos family, LP1, binary64, [-4, 4] in 32 cells, M = 256, N = 10.
# cfg2: d = q = 4 logistic, [-3, 3]^4 in 8^4 cells, M = 128, N = 20, LP1, binary32.
# cfg4: cfg2 with N = 50, M = 32.
# cfg5: d = q = 8 logistic, [-3, 3]^8 in 4^8 = 65536 cells, M = 64, N = 50, LP1, binary32.
CONFIGS: Dict[str, dict] = {
    "cfg1": dict(name="cos d=1 K=32 M=256 N=10 LP1 fp64", d=1, N=10, T=1.0, lo=[-4.0], hi=[4.0],
                 cells=[32], mu=1.0, M=256, basis="LP1", prec="fp64", driver="linear", r=0.05,
                 kappa=0.0, terminal="cos", seed=1, x0=[0.0]),
    "cfg2": dict(name="logistic d=4 K=8^4 M=128 N=20 LP1 fp32", d=4, N=20, T=1.0, lo=[-3.0] * 4,
                 hi=[3.0] * 4, cells=[8] * 4, mu=1.0, M=128, basis="LP1", prec="fp32",
                 driver="logistic", r=0.0, kappa=0.0, terminal="logistic", seed=1, x0=[0.0] * 4),
    "cfg4": dict(name="logistic d=4 K=8^4 M=32 N=50 LP1 fp32", d=4, N=50, T=1.0, lo=[-3.0] * 4,
                 hi=[3.0] * 4, cells=[8] * 4, mu=1.0, M=32, basis="LP1", prec="fp32",
                 driver="logistic", r=0.0, kappa=0.0, terminal="logistic", seed=1, x0=[0.0] * 4),
    "cfg5": dict(name="logistic d=8 K=4^8 M=64 N=50 LP1 fp32", d=8, N=50, T=1.0, lo=[-3.0] * 8,
                 hi=[3.0] * 8, cells=[4] * 8, mu=1.0, M=64, basis="LP1", prec="fp32",
                 driver="logistic", r=0.0, kappa=0.0, terminal="logistic", seed=1, x0=[0.0] * 8),
}


def config(name: str, **overrides) -> dict:
    c = copy.deepcopy(CONFIGS[name])
    c.update(overrides)
    return c


def path_steps(cfg: dict, i_hi: int = None, i_lo: int = 0) -> int:
    """Euler steps simulated by steps i_hi..i_lo: K * M * sum_i (N - i)."""
    K = int(np.prod(cfg["cells"]))
    N = cfg["N"]
    i_hi = N - 1 if i_hi is None else i_hi
    return K * cfg["M"] * sum(N - i for i in range(i_lo, i_hi + 1))


def ragged_batch(n: int = 64, seed: int = 3) -> List[dict]:
    """The ragged batch of d = 2 cos problems: r ~ U[0, 0.2], x0 ~ U[-1, 1]^2,
    C ~ U{16..64} cells per dimension on [-4, 4]^2, M = round(2^U[6, 10]),
    N ~ U{10..50}; sweep seeds 1000 + b.  Drawn with numpy's Philox generator."""
    rng = np.random.Generator(np.random.Philox(seed))
    out = []
    for b in range(n):
        C = int(rng.integers(16, 65))
        out.append(dict(name=f"batch{b}", d=2, N=int(rng.integers(10, 51)), T=1.0,
                        lo=[-4.0, -4.0], hi=[4.0, 4.0], cells=[C, C], mu=1.0,
                        M=int(round(2.0 ** rng.uniform(6.0, 10.0))), basis="LP1", prec="fp32",
                        driver="linear", r=float(rng.uniform(0.0, 0.2)), kappa=0.0,
                        terminal="cos", seed=1000 + b,
                        x0=[float(v) for v in rng.uniform(-1.0, 1.0, 2)]))
    return out
