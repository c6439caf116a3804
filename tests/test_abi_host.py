"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/srmdp.h declares, sizes tables and workspaces, and
rejects invalid arguments before enqueuing anything."""
import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _S():
    import paper_2407_21085_amd as S
    return S


def test_every_declared_function_is_exported():
    S = _S()
    header = open(os.path.join(ROOT, "include", "srmdp.h")).read()
    code = re.sub(r"/\*.*?\*/", "", header, flags=re.S)  # declarations only, not comments
    declared = set(re.findall(r"\b(srmdp_[a-z_]+)\s*\(", code))
    assert declared == set(S.srmdp.EXPORTS)
    for name in declared:
        assert hasattr(S.srmdp.lib, name), name
    assert S.srmdp.lib.srmdp_abi_version() == 108
    # the binding's largest dimension is the header's
    assert int(re.search(r"#define SRMDP_MAX_D (\d+)", header).group(1)) == S.srmdp.MAX_D


def test_table_elems_and_paper_sizes():
    S = _S()
    P = S.Problem(d=1, N=10)
    G = S.Grid([-4.0], [4.0], [32])
    assert S.table_elems(P, G, S.LP1) == 10 * 32 * 2 * 2
    assert S.table_elems(P, G, S.LP0) == 10 * 32 * 2 * 1
    # Table LP0d6_1 footnote: 50 x 14^6 x 7 coefficients, 4 bytes each = 9.81 GiB
    P6 = S.Problem(d=6, N=50)
    G6 = S.Grid([-6.5] * 6, [6.5] * 6, [14] * 6)
    n = S.table_elems(P6, G6, S.LP0)
    assert n == 50 * 14 ** 6 * 7
    assert n * 4 / 2 ** 30 == pytest.approx(9.81, abs=0.01)
    # K = #C^q for rows of the paper's tables
    for d, C, K in [(4, 28, 614656), (11, 4, 4194304), (4, 10, 10000), (19, 2, 524288)]:
        if d <= 16:
            Pd = S.Problem(d=d, N=1)
            assert S.table_elems(Pd, S.Grid([-6.5] * d, [6.5] * d, [C] * d), S.LP0) == K * (1 + d)


def test_workspace_grows_with_the_lookup_rows():
    S = _S()
    G = S.Grid([-3.0] * 4, [3.0] * 4, [8] * 4)
    P = S.Problem(d=4, N=20, driver=S.DRV_LOGISTIC, terminal=S.G_LOGISTIC)
    w32 = S.workspace_bytes(P, G, S.Options(M=128, prec=S.FP32))
    w64 = S.workspace_bytes(P, G, S.Options(M=128, prec=S.FP64))
    # y and sum-z rows: 2 * 5 values padded to 12 (fp32) or 10 (fp64)
    assert w32 >= 20 * 4096 * 12 * 4
    assert w64 >= 20 * 4096 * 10 * 8
    Pc = S.Problem(d=4, N=20, driver=S.DRV_LOGISTIC, terminal=S.G_LOGISTIC, clamp_z=1.0)
    assert S.workspace_bytes(Pc, G, S.Options(M=128, prec=S.FP32)) >= 20 * 4096 * 28 * 4


BAD = [
    ("M below dimension", dict(), dict(M=2)),
    ("d too large", dict(d=20), dict()),
    ("N zero", dict(N=0), dict()),
    ("q != d", dict(q=2), dict()),
    ("unknown driver", dict(driver=7), dict()),
    ("negative clamp", dict(clamp_y=-1.0), dict()),
    ("bad basis", dict(), dict(basis=3)),
    ("bad precision", dict(), dict(prec=5)),
    ("bad lanes", dict(), dict(lanes_per_cube=48)),
    ("bad steps", dict(), dict(step_hi=12)),
    ("steps reversed", dict(), dict(step_hi=2, step_lo=5)),
    ("instance too large", dict(), dict(instance=70000)),
    ("unknown flags", dict(), dict(flags=0x80)),
    ("debug stratum outside the grid", dict(), dict(flags=0x20, debug_step=3, debug_stratum=8)),
    ("debug step outside the sweep", dict(), dict(flags=0x20, debug_step=10, debug_stratum=0)),
]


@pytest.mark.parametrize("name,pkw,okw", BAD, ids=[b[0] for b in BAD])
def test_invalid_arguments_rejected_before_launch(name, pkw, okw):
    S = _S()
    pk = dict(d=3, N=10)
    pk.update(pkw)
    d = pk["d"] if pk["d"] > 0 else 1   # grid arrays as long as the problem's d
    P = S.Problem(**pk)
    G = S.Grid([-1.0] * d, [1.0] * d, [2] * d)
    ok = dict(M=16)
    ok.update(okw)
    O = S.Options(**ok)
    st = S.srmdp._Stats()
    # Non-NULL dummy device pointers: validation must fail before they are used.
    rc = S.srmdp.lib.srmdp_solve(P.c(), G.c(), O.c(), 16, 16, 1 << 40, None, None)
    assert rc == S.srmdp.E_INVALID
    assert S.srmdp.lib.srmdp_last_error().decode() != ""


def test_grid_errors():
    S = _S()
    P = S.Problem(d=2, N=4)
    O = S.Options(M=16)
    for G in [S.Grid([1.0, 0.0], [0.0, 1.0], [2, 2]), S.Grid([0.0, 0.0], [1.0, 1.0], [0, 2]),
              S.Grid([0.0, 0.0], [1.0, 1.0], [2, 2], mu=0.0),
              S.Grid([0.0, 0.0], [1.0, math.inf], [2, 2]),
              S.Grid([0.0, 0.0], [1.0, 1.0], [65536, 65536])]:
        rc = S.srmdp.lib.srmdp_solve(P.c(), G.c(), O.c(), 16, 16, 1 << 40, None, None)
        assert rc == S.srmdp.E_INVALID


def test_workspace_too_small_is_reported():
    S = _S()
    P = S.Problem(d=1, N=4)
    G = S.Grid([-1.0], [1.0], [4])
    O = S.Options(M=16)
    need = S.workspace_bytes(P, G, O)
    rc = S.srmdp.lib.srmdp_solve(P.c(), G.c(), O.c(), 16, 16, need - 1, None, None)
    assert rc == S.srmdp.E_WORKSPACE


def test_mlp_parameter_counts():
    S = _S()
    # (d+1) -> 64 -> 64 -> q: 4804 parameters at d = q = 4, 5320 at d = q = 8
    assert S.mlp_param_count(5, 4) == 4804
    assert S.mlp_param_count(9, 8) == 5320
    assert S.srmdp.lib.srmdp_mlp_param_count(17, 4) == 0
    assert S.srmdp.lib.srmdp_mlp_param_count(4, 17) == 0
    assert S.srmdp.lib.srmdp_mlp_packed_bytes() == 640 + 24 * 1024


CV_BAD = [
    ("cv in binary64", None, dict(cv=1, prec=0), -2),
    ("cv without network", None, dict(cv=1, prec=1, cv_params=None), -1),
    ("unknown cv", None, dict(cv=5, prec=1), -1),
    ("online batch", None, dict(cv=2, prec=1, batch=100), -1),
    ("online updates", None, dict(cv=2, prec=1, updates=0), -1),
    ("online lr", None, dict(cv=2, prec=1, lr=0.0), -1),
    ("cv with global cloud rows", None, dict(cv=1, prec=1, flags=0x10), -2),
]


class _FakeTensor:
    """A stand-in device pointer: validation fails before it is dereferenced."""

    def data_ptr(self):
        return 4096


@pytest.mark.parametrize("name,_unused,kw,status", CV_BAD, ids=[b[0] for b in CV_BAD])
def test_control_variate_options_rejected(name, _unused, kw, status):
    S = _S()
    P = S.Problem(d=3, N=10)
    G = S.Grid([-1.0] * 3, [1.0] * 3, [2] * 3)
    kw = dict(kw)
    tc = S.TrainConfig(updates_per_step=kw.pop("updates", 4), batch=kw.pop("batch", 256),
                       lr=kw.pop("lr", 1e-3))
    params = kw.pop("cv_params", _FakeTensor())
    O = S.Options(M=kw.pop("M", 32), cv_params=params, cv_train=tc, **kw)
    rc = S.srmdp.lib.srmdp_solve(P.c(), G.c(), O.c(), 16, 16, 1 << 40, None, None)
    assert rc == status, S.srmdp.lib.srmdp_last_error().decode()


def test_global_rows_workspace_and_rejections():
    """Streamed clouds: the workspace grows by the strata per launch times the
    global bytes of one stratum (S' and y_{i+1} of each of the M samples in
    the working precision, 256-byte aligned), automatically when a cloud
    exceeds 64 KB of LDS; a negative strata count is rejected."""
    S = _S()
    P = S.Problem(d=1, N=10)
    G = S.Grid([-4.0], [4.0], [32])
    base = S.workspace_bytes(P, G, S.Options(M=40))
    forced = S.workspace_bytes(P, G, S.Options(M=40, flags=S.F_GLOBAL_ROWS, global_rows_strata=8))
    assert forced - base == 8 * 768                         # 40 * 2 * 8 = 640 -> 768
    default = S.workspace_bytes(P, G, S.Options(M=40, flags=S.F_GLOBAL_ROWS))
    assert default - base == 32 * 768                       # every stratum in one launch
    # M = 12000: 480000 bytes of rows per stratum do not fit in LDS: streamed automatically
    big = S.workspace_bytes(P, G, S.Options(M=12000))
    small_lds = S.workspace_bytes(P, G, S.Options(M=12000, global_rows_strata=8))
    assert big - small_lds == 24 * 192000                   # 12000 * 2 * 8
    binary32 = S.workspace_bytes(P, G, S.Options(M=12000, prec=S.FP32, global_rows_strata=8))
    binary32_16 = S.workspace_bytes(P, G, S.Options(M=12000, prec=S.FP32, global_rows_strata=16))
    assert binary32_16 - binary32 == 8 * 96000              # 12000 * 2 * 4
    rc = S.srmdp.lib.srmdp_solve(P.c(), G.c(), S.Options(M=40, global_rows_strata=-1).c(), 16, 16, 1 << 40,
                                 None, None)
    assert rc == -1


def test_high_dimensions_run_binary32_sweeps_only():
    """d = 7, 9, 10 and 11..19 have the global-rows sweep in binary32 with
    look-up modes Y and YZ only: binary64, z truncation (mode Full) and the
    control variate are refused before anything is enqueued; d = 20 is outside
    the ABI."""
    S = _S()
    G = S.Grid([-1.0] * 11, [1.0] * 11, [2] * 11)
    for P, O, status in [
        (S.Problem(d=11, N=3), S.Options(M=40, prec=S.FP64), -2),
        (S.Problem(d=11, N=3, clamp_z=0.5), S.Options(M=40, prec=S.FP32), -2),
        (S.Problem(d=11, N=3), S.Options(M=40, prec=S.FP32, cv=1, cv_params=_FakeTensor()), -2),
    ]:
        rc = S.srmdp.lib.srmdp_solve(P.c(), G.c(), O.c(), 16, 16, 1 << 40, None, None)
        assert rc == status, S.srmdp.lib.srmdp_last_error().decode()
    G19 = S.Grid([-1.0] * 19, [1.0] * 19, [2] * 10 + [1] * 9)
    assert S.workspace_bytes(S.Problem(d=19, N=3), G19, S.Options(M=40, prec=S.FP32)) > 0
    rc = S.srmdp.lib.srmdp_solve(S.Problem(d=19, N=3).c(), G19.c(), S.Options(M=40, prec=S.FP64).c(), 16, 16,
                                 1 << 40, None, None)
    assert rc == -2
    G20 = S.Grid([-1.0] * 20, [1.0] * 20, [2] * 20)
    rc = S.srmdp.lib.srmdp_solve(S.Problem(d=20, N=3).c(), G20.c(), S.Options(M=40, prec=S.FP32).c(), 16, 16,
                                 1 << 40, None, None)
    assert rc == -1


def test_online_workspace_holds_training_state():
    S = _S()
    P = S.Problem(d=4, N=50, driver=S.DRV_LOGISTIC, terminal=S.G_LOGISTIC)
    G = S.Grid([-3.0] * 4, [3.0] * 4, [8] * 4)
    plain = S.workspace_bytes(P, G, S.Options(M=32, prec=S.FP32))
    frozen = S.workspace_bytes(P, G, S.Options(M=32, prec=S.FP32, cv=S.CV_FROZEN,
                                               cv_params=_FakeTensor()))
    tc = S.TrainConfig(updates_per_step=8, batch=512)
    online = S.workspace_bytes(P, G, S.Options(M=32, prec=S.FP32, cv=S.CV_ONLINE,
                                               cv_params=_FakeTensor(), cv_train=tc))
    assert frozen - plain >= 640 + 24 * 1024
    # Adam moments, 8 * 512 pairs of 2 x 16 floats, N * 8 losses, 2 gradient partials
    assert online - frozen >= 2 * 4804 * 4 + 8 * 512 * 32 * 4 + 50 * 8 * 4 + 2 * 4864 * 4


def test_mlp_calls_reject_bad_arguments():
    S = _S()
    lib = S.srmdp.lib
    tc = S.TrainConfig(updates_per_step=2, batch=256).c()
    import ctypes
    # n not a multiple of 64, shape out of range, misaligned pairs
    assert lib.srmdp_mlp_train(5, 4, 16, 16, 16, 0, 4096, 4096, 100, ctypes.byref(tc), 16, None, 16, 1 << 20, None) == -1
    assert lib.srmdp_mlp_train(17, 4, 16, 16, 16, 0, 4096, 4096, 128, ctypes.byref(tc), 16, None, 16, 1 << 20, None) == -1
    assert lib.srmdp_mlp_train(5, 4, 16, 16, 16, 0, 4100, 4096, 128, ctypes.byref(tc), 16, None, 16, 1 << 20, None) == -1
    bad = S.TrainConfig(updates_per_step=2, batch=300).c()
    assert lib.srmdp_mlp_train(5, 4, 16, 16, 16, 0, 4096, 4096, 128, ctypes.byref(bad), 16, None, 16, 1 << 20, None) == -1
    # workspace missing or too small: batch 512 needs 2 partials of (4804 + 1) floats, rounded up to 4864
    tc2 = S.TrainConfig(updates_per_step=2, batch=512).c()
    assert lib.srmdp_mlp_train_workspace_bytes(5, 4, ctypes.byref(tc2)) == 2 * 4864 * 4
    assert lib.srmdp_mlp_train_workspace_bytes(5, 4, ctypes.byref(bad)) == 0
    assert lib.srmdp_mlp_train(5, 4, 16, 16, 16, 0, 4096, 4096, 128, ctypes.byref(tc2), 16, None, None, 0,
                               None) == -1
    assert lib.srmdp_mlp_train(5, 4, 16, 16, 16, 0, 4096, 4096, 128, ctypes.byref(tc2), 16, None, 16,
                               2 * 4864 * 4 - 1, None) == -3
    assert lib.srmdp_mlp_forward(0, 4, 16, 16, 10, 16, None) == -1
    assert lib.srmdp_mlp_forward(5, 4, 16, 16, -1, 16, None) == -1
    assert lib.srmdp_mlp_backward(5, 4, 16, 16, 16, 64, 16, 16, 0, None) == -3
    assert lib.srmdp_mlp_backward_workspace(5, 4, 3000) == 3 * 4804 * 4


def _batch(S, ds=(2, 2), **okw):
    P = [S.Problem(d=d, N=5 + b) for b, d in enumerate(ds)]
    G = [S.Grid([-1.0] * d, [1.0] * d, [3] * d) for d in ds]
    O = [S.Options(M=16, prec=S.FP32, **okw) for _ in ds]
    return P, G, O


def test_batch_workspace_and_rejections():
    S = _S()
    lib = S.srmdp.lib
    P, G, O = _batch(S)
    total = S.workspace_bytes_batch(P, G, O)
    single = sum(S.workspace_bytes(p, g, o) for p, g, o in zip(P, G, O))
    assert total >= single
    for bad, status in [(_batch(S, ds=(2, 3)), -1),                 # different d
                        (_batch(S, step_hi=2), -2),                 # partial sweeps
                        (_batch(S, cv=1, cv_params=_FakeTensor()), -2)]:
        n, Pa, Ga, Oa = S.srmdp._arrays(*bad)
        import ctypes
        ptrs = (ctypes.c_void_p * n)(*([4096] * n))
        rc = lib.srmdp_solve_batch(n, Pa, Ga, Oa, ptrs, 16, 1 << 40, None, None)
        assert rc == status, lib.srmdp_last_error().decode()
    n, Pa, Ga, Oa = S.srmdp._arrays(P, G, O)
    import ctypes
    ptrs = (ctypes.c_void_p * n)(*([4096] * n))
    assert lib.srmdp_solve_batch(0, Pa, Ga, Oa, ptrs, 16, 1 << 40, None, None) == -1
    assert lib.srmdp_solve_batch(n, Pa, Ga, Oa, ptrs, 16, total - 1, None, None) == -3


def test_equal_probability_grid_host_checks():
    """Equal-probability cells: lo and hi may be NULL; the workspace is that of
    an equal-size grid of the same shape (clouds in LDS, or in global memory
    with SRMDP_F_GLOBAL_ROWS); the control variate with z truncation, binary64
    sweeps and z truncation at the dimensions without the LDS kernel, and an
    unknown grid kind are refused before anything is enqueued; a batch may hold equal-probability instances when all of them
    do."""
    import ctypes
    S = _S()
    lib = S.srmdp.lib
    P = S.Problem(d=2, N=4)
    Gp = S.Grid(None, None, [5, 4], 1.3, kind=S.GRID_EQUAL_PROB)
    Gs = S.Grid([-2.0] * 2, [2.0] * 2, [5, 4], 1.3)
    ws_p = S.workspace_bytes(P, Gp, S.Options(M=40))
    assert ws_p == S.workspace_bytes(P, Gs, S.Options(M=40))
    assert (S.workspace_bytes(P, Gp, S.Options(M=40, flags=S.F_GLOBAL_ROWS)) ==
            S.workspace_bytes(P, Gs, S.Options(M=40, flags=S.F_GLOBAL_ROWS)) > ws_p)
    cv = S.Options(M=40, prec=S.FP32, cv=1, cv_params=_FakeTensor())
    Pz = S.Problem(d=2, N=4, clamp_z=0.3)   # z truncation: look-up mode Full
    assert lib.srmdp_solve(Pz.c(), Gp.c(), cv.c(), 16, 16, 1 << 40, None, None) == -2
    # the dimensions without the LDS kernel take equal-probability cells as they
    # take equal-size ones: binary32 sweeps without z truncation
    G7 = S.Grid(None, None, [2] * 7, kind=S.GRID_EQUAL_PROB)
    for prob, opts in ((S.Problem(d=7, N=3), S.Options(M=40, prec=S.FP64)),
                       (S.Problem(d=7, N=3, clamp_z=0.3), S.Options(M=40, prec=S.FP32))):
        rc = lib.srmdp_solve(prob.c(), G7.c(), opts.c(), 16, 16, 1 << 40, None, None)
        assert rc == -2, lib.srmdp_last_error().decode()
    Gbad = S.Grid([-2.0] * 2, [2.0] * 2, [5, 4], 1.3, kind=7)
    assert lib.srmdp_solve(P.c(), Gbad.c(), S.Options(M=40).c(), 16, 16, 1 << 40, None, None) == -1
    Gnull = S.Grid(None, None, [5, 4], 1.3)   # equal size without lo/hi
    assert lib.srmdp_solve(P.c(), Gnull.c(), S.Options(M=40).c(), 16, 16, 1 << 40, None, None) == -1
    # a batch shares the grid kind
    Pb, Gb, Ob = _batch(S)
    Gb[1] = S.Grid(None, None, [3, 3], kind=S.GRID_EQUAL_PROB)
    n, Pa, Ga, Oa = S.srmdp._arrays(Pb, Gb, Ob)
    ptrs = (ctypes.c_void_p * n)(*([4096] * n))
    assert lib.srmdp_solve_batch(n, Pa, Ga, Oa, ptrs, 16, 1 << 40, None, None) == -1


NOALLOC_BAD = [
    ("graph", dict(flags=0x1), -1),
    ("check finite", dict(flags=0x2), -1),
    ("autotune without lanes", dict(flags=0x8), -1),
]


@pytest.mark.parametrize("name,okw,status", NOALLOC_BAD, ids=[b[0] for b in NOALLOC_BAD])
def test_noalloc_refuses_what_allocates_or_synchronises(name, okw, status):
    """srmdp_solve_noalloc refuses graphs, finiteness checks (they copy to the
    host and synchronise) and autotuning before any HIP call."""
    S = _S()
    P = S.Problem(d=2, N=4)
    G = S.Grid([-1.0] * 2, [1.0] * 2, [4, 4])
    O = S.Options(M=16, **okw)
    rc = S.srmdp.lib.srmdp_solve_noalloc(P.c(), G.c(), O.c(), 16, None)
    assert rc == status
    assert "srmdp_solve_noalloc" in S.srmdp.lib.srmdp_last_error().decode()


def test_noalloc_refuses_a_workspace_beyond_its_scratch():
    """The headline workload (d = 8, K = 4^8, N = 50) needs 262 MB of look-up
    rows, more than the 64 MiB array: SRMDP_E_WORKSPACE before any HIP call."""
    S = _S()
    P = S.Problem(d=8, N=50, driver=S.DRV_LOGISTIC, terminal=S.G_LOGISTIC)
    G = S.Grid([-3.0] * 8, [3.0] * 8, [4] * 8)
    O = S.Options(M=64, prec=S.FP32)
    assert S.workspace_bytes(P, G, O) > S.srmdp.NOALLOC_SCRATCH_BYTES
    rc = S.srmdp.lib.srmdp_solve_noalloc(P.c(), G.c(), O.c(), 16, None)
    assert rc == S.srmdp.E_WORKSPACE
    assert "SRMDP_NOALLOC_SCRATCH_BYTES" in S.srmdp.lib.srmdp_last_error().decode()
    header = open(os.path.join(ROOT, "include", "srmdp.h")).read()
    assert re.search(r"#define SRMDP_NOALLOC_SCRATCH_BYTES \(\(size_t\)64 << 20\)", header)
    assert S.srmdp.NOALLOC_SCRATCH_BYTES == 64 << 20


MODEL_BAD = [
    ("empty source", dict(source=""), dict()),
    ("too many parameters", dict(params=[0.0] * 65), dict()),
    ("non-finite parameter", dict(params=[float("nan")]), dict()),
    ("built-in coefficients beside a model", dict(), dict(r=0.5)),
    ("built-in drift beside a model", dict(), dict(b=[0.1, 0.2])),
]


@pytest.mark.parametrize("name,mkw,pkw", MODEL_BAD, ids=[b[0] for b in MODEL_BAD])
def test_model_arguments_rejected_before_compiling(name, mkw, pkw):
    """A problem with its own coefficients is validated before anything is
    compiled or enqueued."""
    S = _S()
    m = dict(source="__device__ void srmdp_b() {}", params=[0.1])
    m.update(mkw)
    P = S.Problem(d=2, N=4, model=S.Model(**m), **pkw)
    G = S.Grid([-1.0] * 2, [1.0] * 2, [2, 2])
    O = S.Options(M=16)
    rc = S.srmdp.lib.srmdp_solve(P.c(), G.c(), O.c(), 16, 16, 1 << 40, None, None)
    assert rc == S.srmdp.E_INVALID
    assert S.srmdp.lib.srmdp_last_error().decode() != ""


def test_model_refused_where_not_supported():
    """Batches and the no-allocation entry point refuse a model before any
    HIP call (compiling one allocates); srmdp_solve refuses a model above
    d = 8 (whole records of (d + 1)^2 coefficients per look-up), with the
    control variate or with the autotuner before compiling it."""
    S = _S()
    src = "__device__ void srmdp_b() {}"
    P = S.Problem(d=2, N=4, model=S.Model(src))
    G = S.Grid([-1.0] * 2, [1.0] * 2, [2, 2])
    O = S.Options(M=16)
    rc = S.srmdp.lib.srmdp_solve_noalloc(P.c(), G.c(), O.c(), 16, None)
    assert rc == S.srmdp.E_INVALID
    assert "model" in S.srmdp.lib.srmdp_last_error().decode()
    lib = S.srmdp.lib
    P9 = S.Problem(d=9, N=3, model=S.Model(src))
    G9 = S.Grid([-1.0] * 9, [1.0] * 9, [2] + [1] * 8)
    assert lib.srmdp_solve(P9.c(), G9.c(), S.Options(M=16, prec=S.FP32).c(), 16, 16, 1 << 40, None,
                           None) == S.srmdp.E_UNSUPPORTED
    assert "d = 1..8" in lib.srmdp_last_error().decode()
    cv = S.Options(M=16, prec=S.FP32, cv=1, cv_params=_FakeTensor())
    assert lib.srmdp_solve(P.c(), G.c(), cv.c(), 16, 16, 1 << 40, None, None) == S.srmdp.E_UNSUPPORTED
    tuned = S.Options(M=16, flags=S.F_AUTOTUNE)
    assert lib.srmdp_solve(P.c(), G.c(), tuned.c(), 16, 16, 1 << 40, None, None) == S.srmdp.E_UNSUPPORTED
