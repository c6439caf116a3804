"""srmdp_solve_noalloc (the sweep with the library's own device scratch array as
workspace) against srmdp_solve with a caller workspace: the same kernels in the
same order, so the tables must agree bit for bit.  Two calls in a row on the
one array, the second with a smaller input, and a control-variate sweep that
trains its network online (its Adam state lives in the scratch array)."""
import sys

import numpy as np
import pytest

import workloads as W
from sides import product_args

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    return torch


def _reference(P, G, Opt):
    """srmdp_solve with a fresh caller workspace filled with 0xFF bytes."""
    import paper_2407_21085_amd as S
    torch = _torch()
    ws = S.srmdp.alloc_workspace(P, G, Opt)
    ws.fill_(0xFF)
    table, _ = S.solve(P, G, Opt, workspace=ws, stats=False)
    torch.cuda.synchronize()
    return table.cpu().numpy()


def _noalloc(P, G, Opt, stream=None):
    import paper_2407_21085_amd as S
    torch = _torch()
    table = S.srmdp.alloc_table(P, G, Opt)
    table.fill_(float("nan"))
    S.solve_noalloc(P, G, Opt, table=table, stream=stream)
    torch.cuda.synchronize()
    return table.cpu().numpy()


CASES = [
    # larger first, then smaller: the second call finds the first one's data in the array
    ("cfg2 fp32 (K = 4096, N = 20)", "cfg2", dict()),
    ("cfg1 fp64 (K = 32, N = 10)", "cfg1", dict()),
    ("cfg2 fp64 N = 6", "cfg2", dict(prec="fp64", N=6)),
    ("d = 3 clamps fp32 N = 5", "cfg1", dict(d=3, N=5, lo=[-2.0] * 3, hi=[2.0] * 3, cells=[3, 4, 2], M=70,
                                          basis="LP1", prec="fp32", driver="logistic", terminal="logistic",
                                          clamp_y=0.7, clamp_z=0.2, x0=[0.0] * 3)),
]


def test_two_calls_in_a_row_match_solve():
    """Every case runs twice through srmdp_solve_noalloc, each after a larger
    one, and each result equals srmdp_solve's bit for bit."""
    torch = _torch()
    stream = torch.cuda.Stream()
    for name, base, kw in CASES:
        cfg = W.config(base, **kw) if base == "cfg2" else dict(W.config(base), **kw)
        P, G, Opt = product_args(cfg)
        _say(f"[gpu] noalloc vs solve: {name}")
        ref = _reference(P, G, Opt)
        with torch.cuda.stream(stream):
            got = _noalloc(P, G, Opt, stream=stream)
        np.testing.assert_array_equal(got, ref)
        got2 = _noalloc(P, G, Opt)
        np.testing.assert_array_equal(got2, ref)


def test_online_control_variate_matches_solve():
    """The online control variate keeps its Adam moments and training pairs
    in the workspace; a second, smaller sweep follows on the same array."""
    import paper_2407_21085_amd as S
    torch = _torch()
    for N in (8, 4):
        cfg = W.config("cfg4", N=N)
        P, G, Opt = product_args(cfg)
        params0 = S.mlp_init(cfg["d"] + 1, cfg["d"], seed=5)
        Opt.cv, Opt.cv_stride = S.CV_ONLINE, 2
        Opt.cv_train = S.TrainConfig(updates_per_step=1, batch=2048, lr=1e-2)
        _say(f"[gpu] noalloc vs solve: online control variate, cfg4 N = {N}")
        Opt.cv_params = params0.clone()
        ref = _reference(P, G, Opt)
        theta_ref = Opt.cv_params.cpu().numpy()
        Opt.cv_params = params0.clone()
        got = _noalloc(P, G, Opt)
        np.testing.assert_array_equal(got, ref)
        np.testing.assert_array_equal(Opt.cv_params.cpu().numpy(), theta_ref)


def test_oversized_request_is_refused_before_launch():
    import paper_2407_21085_amd as S
    cfg = W.config("cfg5")
    P, G, Opt = product_args(cfg)
    assert S.workspace_bytes(P, G, Opt) > S.srmdp.NOALLOC_SCRATCH_BYTES
    table = S.srmdp.alloc_table(P, G, Opt)
    with pytest.raises(S.SrmdpError) as e:
        S.solve_noalloc(P, G, Opt, table=table)
    assert e.value.status == S.srmdp.E_WORKSPACE
