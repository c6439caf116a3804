"""Clouds in global memory: a stratum whose cloud does not fit in a
workgroup's 64 KB of LDS (or any stratum, with SRMDP_F_GLOBAL_ROWS) keeps its
regression inputs and chunk sums in the workspace, and each backward step runs
in launches of global_rows_strata strata.  The arithmetic and its order are
those of the LDS path, so the tables must be bit-identical to it; at large M,
where only this path runs, the tables are held to the FP64 oracle (GPU tests,
through the C ABI)."""
import math
import sys

import numpy as np
import pytest

import test_gpu_parity as TP
import workloads as W
from sides import product_args

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("lanes", [0, 8])
def test_global_rows_bit_identical_to_lds(prec, lanes):
    """K = 3^4 = 81 strata, M = 200 (four chunks of sums, the last ragged):
    one launch per step, launches of 8 strata (the last holds one), and of 24."""
    import paper_2407_21085_amd as S
    cfg = dict(W.config("cfg2"), N=5, cells=[3] * 4, M=200, prec=prec, lanes=lanes)
    ref, st = TP.gpu_table(cfg)
    assert st["step_launches"] == cfg["N"]
    for strata in (0, 8, 24):
        got, st2 = TP.gpu_table(cfg, flags=S.F_GLOBAL_ROWS, global_rows_strata=strata)
        kc = 88 if strata == 0 else strata
        assert st2["step_launches"] == cfg["N"] * math.ceil(81 / kc)
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("d, cells, M, N, lanes", [(6, 3, 200, 3, 0), (6, 3, 200, 3, 64), (8, 2, 64, 4, 0)])
def test_global_rows_bit_identical_to_lds_work_items(d, cells, M, N, lanes):
    """binary32 with more than 64 Gram and z right-hand-side entries (LP1 at
    d = 6: 70, d = 8: 117): the LDS path sums them in work items of three
    entries, the global-memory path one entry per lane; each entry's sum takes
    the same operations in the same order, so the tables are bit-identical
    (d = 6: four chunks of sums at 256 and 64 lanes; d = 8: one chunk)."""
    import paper_2407_21085_amd as S
    cfg = dict(W.config("cfg2", d=d, N=N, lo=[-3.0] * d, hi=[3.0] * d, cells=[cells] * d, M=M),
               prec="fp32", lanes=lanes)
    _say(f"[gpu] global rows against LDS work items: d={d} M={M} lanes={lanes}")
    ref, _ = TP.gpu_table(cfg)
    got, _ = TP.gpu_table(cfg, flags=S.F_GLOBAL_ROWS)
    assert np.isfinite(ref).all()
    np.testing.assert_array_equal(got, ref)


def test_large_cloud_fp64_full_sweep_parity():
    """cfg1 (d = 1, LP1, binary64, K = 32, N = 10) at M = 12000: 480 KB of rows
    per stratum, so the clouds go to global memory by themselves; the whole
    sweep against the oracle at the FP64 bound."""
    cfg = dict(W.config("cfg1"), M=12000)
    gpu, st = TP.gpu_table(cfg)
    assert st["step_launches"] == cfg["N"]
    orc, _ = TP.oracle_table(cfg)
    err = TP.parity(gpu, orc, range(cfg["N"]))
    _say(f"[gpu] cfg1 at M = 12000: parity {err:.3e}")
    assert err <= TP.TOL["fp64"]


def test_large_cloud_fp32_per_step_parity():
    """The d = 4 logistic problem (LP1, binary32, K = 3^4, N = 4) at M = 3000:
    132 KB of rows per stratum, global memory; each step against the oracle's
    step from the same rows, at the FP32 bound.  Strata with a look-up within
    a few ulps of a cell face are compared apart, as in the LDS path's test;
    their share grows with the look-ups per stratum (M (N - i) of them: 8.6 %
    observed here, against about 3 % at M = 128)."""
    cfg = dict(W.config("cfg2"), name="logistic d=4 K=3^4 M=3000 N=4 LP1 fp32", N=4, cells=[3] * 4, M=3000)
    err, excess, share = TP.fp32_step_parity(cfg, [3, 2, 0])
    assert err <= TP.TOL["fp32"]
    assert share < 0.25
    assert excess <= 0.0


def test_global_rows_graph_replays():
    """Launches of 16 strata captured in a hipGraph: three replays, each equal
    to the eager sweep."""
    import paper_2407_21085_amd as S
    torch = TP._torch()
    cfg = dict(W.config("cfg2"), N=5, cells=[3] * 4, M=200)
    P, G, Opt = product_args(cfg, flags=S.F_GLOBAL_ROWS, global_rows_strata=16)
    eager, _ = S.solve(P, G, Opt)
    torch.cuda.synchronize()
    Opt.flags |= S.F_GRAPH
    stream = torch.cuda.Stream()
    table = S.srmdp.alloc_table(P, G, Opt)
    ws = S.srmdp.alloc_workspace(P, G, Opt)
    for rep in range(3):
        _say(f"[gpu] global-rows graph replay {rep}")
        table.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            S.solve(P, G, Opt, table=table, workspace=ws, stream=stream, stats=False)
        torch.cuda.synchronize()
        assert torch.equal(table, eager)
    S.release_graphs()
