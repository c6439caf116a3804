"""Ragged batches and the lanes-per-stratum autotuner on the GPU (called
through the C ABI).

Against the oracle: a binary64 ragged batch, every instance over its whole
sweep at 1e-9; and instances of the 64-instance binary32 workload (the
smallest, the largest M, the largest N) step by step, each step against the
oracle's step run from the batch's own rows above it, at 2e-4 plus the
oracle's face-flip bound.

Self-consistency: a batched sweep computes every stratum group exactly as the
per-instance sweep does (same draws, same sums in the same order), so each
table of a batch must also equal, bit for bit, the table srmdp_solve returns
for that instance alone with the same lanes per stratum.  The same holds
across lane counts, which is what lets the autotuner change them freely.
"""
import sys

import numpy as np
import pytest

import oracle as O
import test_gpu_parity as TP
import workloads as W
from sides import oracle_problem, product_args

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    return torch


def _small_ragged(prec, n=10, seed=5):
    """Ragged d = 2 cos instances: K from 4 to 100 strata, M from 8 to 300 (8 to
    256 lanes per stratum), N from 3 to 12, different rates, seeds and instance
    tags."""
    rng = np.random.default_rng(seed)
    cfgs = []
    for b in range(n):
        C = int(rng.integers(2, 11))
        cfgs.append(dict(name=f"r{b}", d=2, N=int(rng.integers(3, 13)), T=1.0, lo=[-3.0, -3.0],
                         hi=[3.0, 3.0], cells=[C, int(rng.integers(2, 11))], mu=1.0,
                         M=int(rng.choice([8, 16, 24, 40, 64, 100, 300])), basis="LP1", prec=prec,
                         driver="linear", r=float(rng.uniform(0, 0.3)), kappa=float(rng.uniform(0, 0.3)),
                         terminal="cos", seed=100 + b, instance=b % 3))
    return cfgs


def _args(cfgs):
    P, G, O = [], [], []
    for c in cfgs:
        p, g, o = product_args(c)
        P.append(p)
        G.append(g)
        O.append(o)
    return P, G, O


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ragged_batch_equals_individual_sweeps(prec):
    import paper_2407_21085_amd as S
    torch = _torch()
    cfgs = _small_ragged(prec)
    P, G, O = _args(cfgs)
    _say(f"[gpu] ragged batch of {len(cfgs)} ({prec})")
    tables, stats = S.solve_batch(P, G, O)
    torch.cuda.synchronize()
    assert all(s["step_launches"] == max(c["N"] for c in cfgs) for s in stats)
    for c, p, g, o, t, st in zip(cfgs, P, G, O, tables, stats):
        o.lanes_per_cube = st["lanes_per_cube"]
        ref, _ = S.solve(p, g, o)
        torch.cuda.synchronize()
        assert torch.equal(t, ref), c["name"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_equal_probability_batch_equals_individual_sweeps(prec):
    """A ragged batch on equal-probability cells (every instance of the batch
    on that grid) gives each instance's own table bit for bit."""
    import paper_2407_21085_amd as S
    torch = _torch()
    cfgs = [dict(c, lo=None, hi=None, grid_kind=1, mu=0.8 + 0.1 * b)
            for b, c in enumerate(_small_ragged(prec, n=6, seed=9))]
    P, G, O = _args(cfgs)
    _say(f"[gpu] equal-probability ragged batch of {len(cfgs)} ({prec})")
    tables, stats = S.solve_batch(P, G, O)
    torch.cuda.synchronize()
    for c, p, g, o, t, st in zip(cfgs, P, G, O, tables, stats):
        o.lanes_per_cube = st["lanes_per_cube"]
        ref, _ = S.solve(p, g, o)
        torch.cuda.synchronize()
        assert torch.equal(t, ref), c["name"]


def test_ragged_batch_graph_replays():
    import paper_2407_21085_amd as S
    torch = _torch()
    cfgs = _small_ragged("fp32", n=7, seed=9)
    P, G, O = _args(cfgs)
    eager, _ = S.solve_batch(P, G, O)
    for o in O:
        o.flags |= S.F_GRAPH
    stream = torch.cuda.Stream()
    ws = torch.empty(S.workspace_bytes_batch(P, G, O), dtype=torch.uint8, device="cuda")
    tables = [torch.zeros_like(t) for t in eager]
    for rep in range(3):
        for t in tables:
            t.zero_()
        torch.cuda.synchronize()
        _say(f"[gpu] ragged batch graph replay {rep}")
        with torch.cuda.stream(stream):
            S.solve_batch(P, G, O, tables=tables, workspace=ws, stream=stream, stats=False)
        torch.cuda.synchronize()
        for a, b in zip(tables, eager):
            assert torch.equal(a, b)
    S.release_graphs()


def test_full_ragged_batch_workload():
    """The 64-instance ragged batch (K 16^2..64^2, M 64..1024, N 10..50, FP32):
    four of its instances against their individual sweeps, and the whole
    batch finite."""
    import paper_2407_21085_amd as S
    torch = _torch()
    cfgs = W.ragged_batch()
    P, G, O = _args(cfgs)
    _say("[gpu] 64-instance ragged batch")
    tables, stats = S.solve_batch(P, G, O)
    torch.cuda.synchronize()
    _say(f"[gpu]   batch {stats[0]['ms_total']:.2f} ms for {sum(s['path_steps'] for s in stats):.3e} path-steps")
    assert all(bool(torch.isfinite(t).all()) for t in tables)
    for b in (0, 17, 40, 63):
        O[b].lanes_per_cube = stats[b]["lanes_per_cube"]
        ref, _ = S.solve(P[b], G[b], O[b])
        torch.cuda.synchronize()
        assert torch.equal(tables[b], ref), b


def test_autotuner_picks_a_candidate_and_keeps_results():
    import paper_2407_21085_amd as S
    torch = _torch()
    cfg = W.config("cfg2")
    P, G, O = product_args(cfg)
    _say("[gpu] autotune cfg2")
    lanes, ms = S.tune_lanes(P, G, O)
    _say(f"[gpu]   lanes {lanes}, ms per launch {ms}")
    cand = [8, 16, 32, 64, 128, 256]
    assert lanes in cand
    assert ms[cand.index(lanes)] == min(m for m in ms if m >= 0)
    assert ms[cand.index(8)] > 0 and ms[cand.index(128)] > 0   # M = 128: up to 128 lanes tried
    assert ms[cand.index(256)] == -1.0
    O.flags |= S.F_AUTOTUNE
    tuned, st = S.solve(P, G, O)
    assert st["lanes_per_cube"] == lanes
    O.flags &= ~S.F_AUTOTUNE
    O.lanes_per_cube = 8 if lanes != 8 else 64
    other, _ = S.solve(P, G, O)
    torch.cuda.synchronize()
    assert torch.equal(tuned, other)


def test_autotuned_batch_matches_individual_sweeps():
    import paper_2407_21085_amd as S
    torch = _torch()
    cfgs = _small_ragged("fp32", n=5, seed=21)
    P, G, O = _args(cfgs)
    for o in O:
        o.flags |= S.F_AUTOTUNE
    tables, stats = S.solve_batch(P, G, O)
    torch.cuda.synchronize()
    for p, g, o, t, st in zip(P, G, O, tables, stats):
        assert st["lanes_per_cube"] in (8, 16, 32, 64, 128, 256)
        o.flags &= ~S.F_AUTOTUNE
        ref, _ = S.solve(p, g, o)
        torch.cuda.synchronize()
        assert torch.equal(t, ref)


def test_ragged_batch_fp64_against_oracle():
    """Ten binary64 instances (K 4..100, M 8..300, N 3..12, different rates,
    seeds and instance tags) in one batch: every table, whole sweep, within
    1e-9 of the oracle's."""
    import paper_2407_21085_amd as S
    torch = _torch()
    cfgs = _small_ragged("fp64")
    P, G, Ob = _args(cfgs)
    _say(f"[gpu] binary64 ragged batch of {len(cfgs)} against the oracle")
    tables, _ = S.solve_batch(P, G, Ob)
    torch.cuda.synchronize()
    worst = 0.0
    for c, t in zip(cfgs, tables):
        orc, _ = O.solve(oracle_problem(c))
        err = TP.parity(t.cpu().numpy(), orc, range(c["N"]))
        worst = max(worst, err)
        assert err <= TP.TOL["fp64"], c["name"]
    _say(f"[gpu] worst instance parity {worst:.3e}")


def test_full_ragged_batch_instances_against_oracle():
    """The 64-instance binary32 ragged batch (K 16^2..64^2, M 64..1024,
    N 10..50) in one batched sweep; its smallest instance, the one with the
    largest M and the one with the largest N, each at steps N-1, N/2 and 0
    against the oracle's step from the batch's own rows above it."""
    import paper_2407_21085_amd as S
    torch = _torch()
    cfgs = W.ragged_batch()
    P, G, Ob = _args(cfgs)
    _say(f"[gpu] the {len(cfgs)}-instance ragged batch")
    tables, _ = S.solve_batch(P, G, Ob)
    torch.cuda.synchronize()

    def work(c):
        return int(np.prod(c["cells"])) * c["M"] * c["N"] * (c["N"] + 1) // 2

    picks = {min(range(len(cfgs)), key=lambda b: work(cfgs[b])),
             max(range(len(cfgs)), key=lambda b: cfgs[b]["M"]),
             max(range(len(cfgs)), key=lambda b: (cfgs[b]["N"], -work(cfgs[b])))}
    for b in sorted(picks):
        c = cfgs[b]
        gpu = tables[b].double().cpu().numpy()
        steps = sorted({c["N"] - 1, c["N"] // 2, 0}, reverse=True)
        for i in steps:
            _say(f"[gpu] {c['name']} (K = {int(np.prod(c['cells']))}, M = {c['M']}, N = {c['N']}): "
                 f"oracle step {i} from the batch's rows")
            orc, flags, bound = TP._oracle_with_flags(c, i, i, 2e-6, table=gpu.copy())
            err, excess = TP.bounded_parity(gpu, orc, bound, [i], flags, TP.TOL["fp32"])
            assert err <= TP.TOL["fp32"], (c["name"], i)
            assert excess <= 0.0, (c["name"], i)
