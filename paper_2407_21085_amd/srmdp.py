"""Python binding of libsrmdp.so (include/srmdp.h): argument marshalling only.

Every step of the sweep runs in the library's HIP kernels.  PyTorch provides
device memory (tensors) and streams; nothing here computes any part of the
method.  Importing this module fails loudly if the library is not built.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsrmdp.so")

OK, E_INVALID, E_UNSUPPORTED, E_WORKSPACE, E_HIP, E_NUMERIC = 0, -1, -2, -3, -4, -5
LP0, LP1 = 0, 1
FP64, FP32 = 0, 1
DRV_LINEAR, DRV_LOGISTIC = 0, 1
G_COS_SUM, G_LOGISTIC = 0, 1
F_GRAPH, F_CHECK_FINITE, F_CV_CENTER_Z, F_AUTOTUNE, F_GLOBAL_ROWS = 0x1, 0x2, 0x4, 0x8, 0x10
F_DEBUG_SINGULAR = 0x20
GRID_EQUAL_SIZE, GRID_EQUAL_PROB = 0, 1
CV_NONE, CV_FROZEN, CV_ONLINE = 0, 1, 2
MAX_D = 19   # SRMDP_MAX_D of include/srmdp.h
MLP_HIDDEN = 64


class SrmdpError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"srmdp status {status}: {message}")
        self.status = status


class _Model(ctypes.Structure):
    _fields_ = [("source", ctypes.c_char_p), ("params", ctypes.POINTER(ctypes.c_double)),
                ("n_params", ctypes.c_int32)]


class _Problem(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32), ("q", ctypes.c_int32),
        ("T", ctypes.c_double), ("N", ctypes.c_int32),
        ("b", ctypes.POINTER(ctypes.c_double)), ("sigma", ctypes.POINTER(ctypes.c_double)),
        ("driver", ctypes.c_int32), ("terminal", ctypes.c_int32),
        ("r", ctypes.c_double), ("kappa", ctypes.c_double),
        ("clamp_y", ctypes.c_double), ("clamp_z", ctypes.c_double),
        ("b_lin", ctypes.POINTER(ctypes.c_double)),
        ("sigma_lin", ctypes.POINTER(ctypes.c_double)),
        ("model", ctypes.POINTER(_Model)),
    ]


class _Grid(ctypes.Structure):
    _fields_ = [
        ("lo", ctypes.POINTER(ctypes.c_double)), ("hi", ctypes.POINTER(ctypes.c_double)),
        ("cells", ctypes.POINTER(ctypes.c_int32)), ("mu", ctypes.c_double),
        ("kind", ctypes.c_int32),
    ]


class _TrainConfig(ctypes.Structure):
    _fields_ = [
        ("updates_per_step", ctypes.c_int32), ("batch", ctypes.c_int32),
        ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
        ("eps", ctypes.c_float),
    ]


class _Options(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int32), ("basis", ctypes.c_int32), ("prec", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("instance", ctypes.c_uint32),
        ("step_hi", ctypes.c_int32), ("step_lo", ctypes.c_int32),
        ("lanes_per_cube", ctypes.c_int32), ("flags", ctypes.c_uint32),
        ("face_flags", ctypes.c_void_p), ("face_eps", ctypes.c_double),
        ("cv", ctypes.c_int32), ("cv_params", ctypes.c_void_p), ("cv_train", _TrainConfig),
        ("cv_stride", ctypes.c_int32), ("global_rows_strata", ctypes.c_int32),
        ("debug_step", ctypes.c_int32), ("debug_stratum", ctypes.c_uint32),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("singular_cubes", ctypes.c_uint64), ("path_steps", ctypes.c_uint64),
        ("ms_total", ctypes.c_float), ("ms_steps", ctypes.c_float),
        ("step_launches", ctypes.c_int32), ("lanes_per_cube", ctypes.c_int32),
        ("near_face_paths", ctypes.c_uint64),
        ("cv_loss_first", ctypes.c_float), ("cv_loss_last", ctypes.c_float),
    ]


EXPORTS = ("srmdp_table_elems", "srmdp_workspace_bytes", "srmdp_solve", "srmdp_eval",
           "srmdp_root", "srmdp_draw", "srmdp_tune_lanes", "srmdp_workspace_bytes_batch",
           "srmdp_solve_batch", "srmdp_cv_pairs", "srmdp_mlp_param_count",
           "srmdp_mlp_packed_bytes", "srmdp_mlp_init", "srmdp_mlp_pack", "srmdp_mlp_forward",
           "srmdp_mlp_backward_workspace", "srmdp_mlp_backward", "srmdp_mlp_train_workspace_bytes",
           "srmdp_mlp_train",
           "srmdp_solve_noalloc", "srmdp_to_raw_basis", "srmdp_release_graphs", "srmdp_last_error",
           "srmdp_abi_version")


def _load():
    # SRMDP_LIBRARY names another build of this library (an instrumented one)
    path = os.environ.get("SRMDP_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2407_21085_amd.build`")
    # PyTorch ships its own HIP runtime.  Loading torch first makes the library
    # bind to that same runtime (same soname), so one process holds one HIP
    # runtime and the library can work on torch's tensors and streams.
    import torch  # noqa: F401
    L = ctypes.CDLL(path)
    P, G, O, S = (ctypes.POINTER(_Problem), ctypes.POINTER(_Grid), ctypes.POINTER(_Options),
                  ctypes.POINTER(_Stats))
    vp, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    L.srmdp_table_elems.argtypes = [P, G, ctypes.c_int32]
    L.srmdp_table_elems.restype = ctypes.c_size_t
    L.srmdp_workspace_bytes.argtypes = [P, G, O]
    L.srmdp_workspace_bytes.restype = ctypes.c_size_t
    L.srmdp_solve.argtypes = [P, G, O, vp, vp, ctypes.c_size_t, S, vp]
    L.srmdp_solve.restype = ctypes.c_int
    L.srmdp_eval.argtypes = [P, G, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int32, vp,
                             ctypes.c_int64, vp, vp, vp]
    L.srmdp_eval.restype = ctypes.c_int
    L.srmdp_to_raw_basis.argtypes = [P, G, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
    L.srmdp_to_raw_basis.restype = ctypes.c_int
    L.srmdp_root.argtypes = [P, G, O, vp, dp, ctypes.c_int32, dp, dp, vp, ctypes.c_size_t, vp]
    L.srmdp_root.restype = ctypes.c_int
    L.srmdp_draw.argtypes = [P, G, O, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32,
                             ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int32,
                             vp, vp]
    L.srmdp_draw.restype = ctypes.c_int
    i32, i64, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.srmdp_solve_noalloc.argtypes = [P, G, O, vp, vp]
    L.srmdp_solve_noalloc.restype = ctypes.c_int
    L.srmdp_tune_lanes.argtypes = [P, G, O, vp, vp, sz, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float), vp]
    L.srmdp_tune_lanes.restype = ctypes.c_int
    L.srmdp_workspace_bytes_batch.argtypes = [i32, P, G, O]
    L.srmdp_workspace_bytes_batch.restype = sz
    L.srmdp_solve_batch.argtypes = [i32, P, G, O, ctypes.POINTER(vp), vp, sz, S, vp]
    L.srmdp_solve_batch.restype = ctypes.c_int
    L.srmdp_cv_pairs.argtypes = [P, G, O, vp, i32, i64, vp, vp, vp, sz, vp]
    L.srmdp_cv_pairs.restype = ctypes.c_int
    L.srmdp_mlp_param_count.argtypes = [i32, i32]
    L.srmdp_mlp_param_count.restype = i64
    L.srmdp_mlp_packed_bytes.argtypes = []
    L.srmdp_mlp_packed_bytes.restype = sz
    L.srmdp_mlp_init.argtypes = [i32, i32, ctypes.c_uint64, i32, vp, vp]
    L.srmdp_mlp_init.restype = ctypes.c_int
    L.srmdp_mlp_pack.argtypes = [i32, i32, vp, vp, vp]
    L.srmdp_mlp_pack.restype = ctypes.c_int
    L.srmdp_mlp_forward.argtypes = [i32, i32, vp, vp, i64, vp, vp]
    L.srmdp_mlp_forward.restype = ctypes.c_int
    L.srmdp_mlp_backward_workspace.argtypes = [i32, i32, i64]
    L.srmdp_mlp_backward_workspace.restype = sz
    L.srmdp_mlp_backward.argtypes = [i32, i32, vp, vp, vp, i64, vp, vp, sz, vp]
    L.srmdp_mlp_backward.restype = ctypes.c_int
    L.srmdp_mlp_train_workspace_bytes.argtypes = [i32, i32, ctypes.POINTER(_TrainConfig)]
    L.srmdp_mlp_train_workspace_bytes.restype = sz
    L.srmdp_mlp_train.argtypes = [i32, i32, vp, vp, vp, i64, vp, vp, i64,
                                  ctypes.POINTER(_TrainConfig), vp, vp, vp, sz, vp]
    L.srmdp_mlp_train.restype = ctypes.c_int
    L.srmdp_release_graphs.argtypes = []
    L.srmdp_release_graphs.restype = None
    L.srmdp_last_error.argtypes = []
    L.srmdp_last_error.restype = ctypes.c_char_p
    L.srmdp_abi_version.argtypes = []
    L.srmdp_abi_version.restype = ctypes.c_int32
    return L


lib = _load()


def _check(status: int) -> None:
    if status != OK:
        raise SrmdpError(status, lib.srmdp_last_error().decode())


def _darr(v: Sequence[float]):
    return (ctypes.c_double * len(v))(*[float(a) for a in v])


@dataclass
class Model:
    """A problem's own coefficients (srmdp_model): HIP device source defining
    srmdp_b, srmdp_sigma_dw, srmdp_f and srmdp_g on `srmdp_real` (the drift,
    the diffusion applied to dW, the driver and the terminal condition),
    compiled at run time, and its parameters p[0..n-1]."""
    source: str
    params: Sequence[float] = ()


@dataclass
class Problem:
    """Problem data of eq. (fbsde)-(eds): drift b + diag(b_lin) x, diffusion
    sigma + diag(sigma_lin) x."""
    d: int
    N: int
    T: float = 1.0
    q: Optional[int] = None
    driver: int = DRV_LINEAR
    terminal: int = G_COS_SUM
    r: float = 0.0
    kappa: float = 0.0
    clamp_y: float = math.inf
    clamp_z: float = math.inf
    b: Optional[Sequence[float]] = None
    sigma: Optional[Sequence[float]] = None
    b_lin: Optional[Sequence[float]] = None   # drift b_l + b_lin_l x_l (Ornstein-Uhlenbeck)
    sigma_lin: Optional[Sequence[float]] = None   # diffusion sigma + diag(sigma_lin) x
    model: Optional[Model] = None                 # own coefficients compiled at run time
    _keep: list = field(default_factory=list, repr=False)

    def c(self) -> _Problem:
        q = self.d if self.q is None else self.q
        s = _Problem(self.d, q, self.T, self.N, None, None, self.driver, self.terminal, self.r,
                     self.kappa, self.clamp_y, self.clamp_z)
        self._keep = []
        if self.b is not None:
            a = _darr(self.b)
            self._keep.append(a)
            s.b = ctypes.cast(a, ctypes.POINTER(ctypes.c_double))
        if self.sigma is not None:
            a = _darr(self.sigma)
            self._keep.append(a)
            s.sigma = ctypes.cast(a, ctypes.POINTER(ctypes.c_double))
        if self.b_lin is not None:
            a = _darr(self.b_lin)
            self._keep.append(a)
            s.b_lin = ctypes.cast(a, ctypes.POINTER(ctypes.c_double))
        if self.sigma_lin is not None:
            a = _darr(self.sigma_lin)
            self._keep.append(a)
            s.sigma_lin = ctypes.cast(a, ctypes.POINTER(ctypes.c_double))
        if self.model is not None:
            src = self.model.source.encode()
            prm = _darr(self.model.params) if len(self.model.params) else None
            m = _Model(src, ctypes.cast(prm, ctypes.POINTER(ctypes.c_double)) if prm is not None else None,
                       len(self.model.params))
            self._keep += [src, prm, m]
            s.model = ctypes.pointer(m)
        return s


@dataclass
class Grid:
    """Stratification with the logistic sampling law: equal-size cells of
    [lo, hi) (GRID_EQUAL_SIZE), or cells cut at the logistic quantiles so that
    every cube has probability 1/K (GRID_EQUAL_PROB; lo and hi unused)."""
    lo: Optional[Sequence[float]]
    hi: Optional[Sequence[float]]
    cells: Sequence[int]
    mu: float = 1.0
    kind: int = GRID_EQUAL_SIZE
    _keep: list = field(default_factory=list, repr=False)

    @property
    def K(self) -> int:
        k = 1
        for c in self.cells:
            k *= int(c)
        return k

    def c(self) -> _Grid:
        dp = ctypes.POINTER(ctypes.c_double)
        lo = _darr(self.lo) if self.lo is not None else None
        hi = _darr(self.hi) if self.hi is not None else None
        cells = (ctypes.c_int32 * len(self.cells))(*[int(c) for c in self.cells])
        self._keep = [lo, hi, cells]
        return _Grid(ctypes.cast(lo, dp) if lo is not None else None,
                     ctypes.cast(hi, dp) if hi is not None else None,
                     ctypes.cast(cells, ctypes.POINTER(ctypes.c_int32)), self.mu, int(self.kind))


@dataclass
class TrainConfig:
    """Online training of the control-variate network (Adam)."""
    updates_per_step: int = 16
    batch: int = 512
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8

    def c(self) -> _TrainConfig:
        return _TrainConfig(self.updates_per_step, self.batch, self.lr, self.beta1, self.beta2,
                            self.eps)


@dataclass
class Options:
    M: int
    basis: int = LP1
    prec: int = FP64
    seed: int = 1
    instance: int = 0
    step_hi: int = -1
    step_lo: int = -1
    lanes_per_cube: int = 0
    flags: int = 0
    face_flags: object = None   # device uint8 tensor [N, K] or None
    face_eps: float = 0.0
    cv: int = CV_NONE
    cv_params: object = None    # device float32 tensor [mlp_param_count(d+1, q)] or None
    cv_train: TrainConfig = field(default_factory=TrainConfig)
    cv_stride: int = 1
    global_rows_strata: int = 0
    debug_step: int = 0         # F_DEBUG_SINGULAR: step and stratum of the zeroed Gram
    debug_stratum: int = 0

    def c(self) -> _Options:
        ptr = self.face_flags.data_ptr() if self.face_flags is not None else None
        cvp = self.cv_params.data_ptr() if self.cv_params is not None else None
        return _Options(self.M, self.basis, self.prec, self.seed, self.instance, self.step_hi,
                        self.step_lo, self.lanes_per_cube, self.flags, ptr, self.face_eps,
                        self.cv, cvp, self.cv_train.c(), self.cv_stride, self.global_rows_strata,
                        self.debug_step, self.debug_stratum)


def table_elems(problem: Problem, grid: Grid, basis: int) -> int:
    return int(lib.srmdp_table_elems(problem.c(), grid.c(), basis))


def workspace_bytes(problem: Problem, grid: Grid, opts: Options) -> int:
    n = int(lib.srmdp_workspace_bytes(problem.c(), grid.c(), opts.c()))
    if n == 0:
        raise SrmdpError(E_INVALID, lib.srmdp_last_error().decode())
    return n


def _torch():
    import torch
    return torch


def _stream_ptr(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) or None


def table_shape(problem: Problem, grid: Grid, basis: int):
    nb = problem.d + 1 if basis == LP1 else 1
    q = problem.d if problem.q is None else problem.q
    return (problem.N, grid.K, 1 + q, nb)


def alloc_table(problem: Problem, grid: Grid, opts: Options, device="cuda"):
    torch = _torch()
    dtype = torch.float32 if opts.prec == FP32 else torch.float64
    return torch.zeros(table_shape(problem, grid, opts.basis), dtype=dtype, device=device)


def alloc_workspace(problem: Problem, grid: Grid, opts: Options, device="cuda"):
    torch = _torch()
    return torch.empty(workspace_bytes(problem, grid, opts), dtype=torch.uint8, device=device)


def solve(problem: Problem, grid: Grid, opts: Options, table=None, workspace=None, stream=None,
          stats: bool = True):
    """Algorithm SRMDP (steps opts.step_hi .. opts.step_lo).  Returns
    (table, stats dict or None)."""
    if table is None:
        table = alloc_table(problem, grid, opts)
    if workspace is None:
        workspace = alloc_workspace(problem, grid, opts)
    st = _Stats()
    rc = lib.srmdp_solve(problem.c(), grid.c(), opts.c(), table.data_ptr(), workspace.data_ptr(),
                         workspace.numel(), ctypes.byref(st) if stats else None,
                         _stream_ptr(stream))
    _check(rc)
    out = None
    if stats:
        out = {"singular_cubes": int(st.singular_cubes), "path_steps": int(st.path_steps),
               "ms_total": float(st.ms_total), "ms_steps": float(st.ms_steps),
               "step_launches": int(st.step_launches), "lanes_per_cube": int(st.lanes_per_cube),
               "near_face_paths": int(st.near_face_paths),
               "cv_loss_first": float(st.cv_loss_first), "cv_loss_last": float(st.cv_loss_last)}
    return table, out


NOALLOC_SCRATCH_BYTES = 64 << 20   # SRMDP_NOALLOC_SCRATCH_BYTES


def solve_noalloc(problem: Problem, grid: Grid, opts: Options, table=None, stream=None):
    """srmdp_solve_noalloc: the sweep with the library's own device scratch
    array as workspace (no allocation by the library; asynchronous, no stats).
    Returns the table (allocated here by torch only when none is given)."""
    if table is None:
        table = alloc_table(problem, grid, opts)
    _check(lib.srmdp_solve_noalloc(problem.c(), grid.c(), opts.c(), table.data_ptr(), _stream_ptr(stream)))
    return table


def evaluate(problem: Problem, grid: Grid, basis: int, prec: int, table, i: int, x, stream=None):
    """Fitted, truncated y_i and z_i at the rows of x (device float64 [n, d])."""
    torch = _torch()
    x = x.to(dtype=torch.float64).contiguous()
    n = x.shape[0]
    q = problem.d if problem.q is None else problem.q
    y = torch.empty(n, dtype=torch.float64, device=x.device)
    z = torch.empty((n, q), dtype=torch.float64, device=x.device)
    _check(lib.srmdp_eval(problem.c(), grid.c(), basis, prec, table.data_ptr(), i, x.data_ptr(),
                          n, y.data_ptr(), z.data_ptr(), _stream_ptr(stream)))
    return y, z


def to_raw_basis(problem: Problem, grid: Grid, basis: int, prec: int, table, out=None, stream=None):
    """The table's coefficients on the paper's raw basis (1, x_1..x_d) (srmdp_to_raw_basis);
    out may be table itself."""
    torch = _torch()
    out = torch.empty_like(table) if out is None else out
    _check(lib.srmdp_to_raw_basis(problem.c(), grid.c(), basis, prec, table.data_ptr(), out.data_ptr(),
                                  _stream_ptr(stream)))
    return out


def root(problem: Problem, grid: Grid, opts: Options, table, x0: Sequence[float], M_root: int,
         workspace=None, stream=None):
    """ROOT read-out of y(0, x0), z(0, x0) (synchronises the stream)."""
    if workspace is None:
        workspace = alloc_workspace(problem, grid, opts, device=table.device)
    q = problem.d if problem.q is None else problem.q
    x0a = _darr(x0)
    y0 = ctypes.c_double(0.0)
    z0 = (ctypes.c_double * q)()
    _check(lib.srmdp_root(problem.c(), grid.c(), opts.c(), table.data_ptr(),
                          ctypes.cast(x0a, ctypes.POINTER(ctypes.c_double)), M_root,
                          ctypes.byref(y0), ctypes.cast(z0, ctypes.POINTER(ctypes.c_double)),
                          workspace.data_ptr(), workspace.numel(), _stream_ptr(stream)))
    return float(y0.value), [float(v) for v in z0]


def draw(problem: Problem, grid: Grid, opts: Options, kind: int, i: int, k0: int, nk: int,
         m0: int, nm: int, count: int, stream=None):
    """The sweep's random inputs (kind 0 uniforms, 1 normals, 2 start points)."""
    torch = _torch()
    out = torch.empty((nk, nm, count), dtype=torch.float64, device="cuda")
    _check(lib.srmdp_draw(problem.c(), grid.c(), opts.c(), kind, i, k0, nk, m0, nm, count,
                          out.data_ptr(), _stream_ptr(stream)))
    return out


def cv_pairs(problem: Problem, grid: Grid, opts: Options, table, i: int, n: int, workspace=None,
             stream=None):
    """Training pairs of the online control variate after step i:
    (x16 [n, 16], z16 [n, 16]) float32 device tensors."""
    torch = _torch()
    if workspace is None:
        workspace = alloc_workspace(problem, grid, opts, device=table.device)
    x16 = torch.empty((n, 16), dtype=torch.float32, device=table.device)
    z16 = torch.empty((n, 16), dtype=torch.float32, device=table.device)
    _check(lib.srmdp_cv_pairs(problem.c(), grid.c(), opts.c(), table.data_ptr(), i, n,
                              x16.data_ptr(), z16.data_ptr(), workspace.data_ptr(),
                              workspace.numel(), _stream_ptr(stream)))
    return x16, z16


def mlp_param_count(n_in: int, n_out: int) -> int:
    n = int(lib.srmdp_mlp_param_count(n_in, n_out))
    if n == 0:
        raise SrmdpError(E_INVALID, f"network shape {n_in} -> {n_out} is not supported")
    return n


def mlp_init(n_in: int, n_out: int, seed: int, zero_output_layer: bool = False, stream=None):
    """Glorot-uniform parameters (float32 device tensor)."""
    torch = _torch()
    p = torch.empty(mlp_param_count(n_in, n_out), dtype=torch.float32, device="cuda")
    _check(lib.srmdp_mlp_init(n_in, n_out, seed, int(zero_output_layer), p.data_ptr(),
                              _stream_ptr(stream)))
    return p


def mlp_pack(n_in: int, n_out: int, params, stream=None):
    torch = _torch()
    packed = torch.empty(int(lib.srmdp_mlp_packed_bytes()), dtype=torch.uint8, device=params.device)
    _check(lib.srmdp_mlp_pack(n_in, n_out, params.data_ptr(), packed.data_ptr(), _stream_ptr(stream)))
    return packed


def mlp_forward(n_in: int, n_out: int, packed, x, stream=None):
    """z_theta(x) for x float32 [n, n_in] on the device."""
    torch = _torch()
    x = x.to(dtype=torch.float32).contiguous()
    y = torch.empty((x.shape[0], n_out), dtype=torch.float32, device=x.device)
    _check(lib.srmdp_mlp_forward(n_in, n_out, packed.data_ptr(), x.data_ptr(), x.shape[0],
                                 y.data_ptr(), _stream_ptr(stream)))
    return y


def mlp_backward(n_in: int, n_out: int, packed, x, dy, stream=None):
    """Gradient of sum_s <dy_s, z_theta(x_s)> with respect to the parameters."""
    torch = _torch()
    x = x.to(dtype=torch.float32).contiguous()
    dy = dy.to(dtype=torch.float32).contiguous()
    n = x.shape[0]
    grad = torch.empty(mlp_param_count(n_in, n_out), dtype=torch.float32, device=x.device)
    ws = torch.empty(int(lib.srmdp_mlp_backward_workspace(n_in, n_out, n)), dtype=torch.uint8,
                     device=x.device)
    _check(lib.srmdp_mlp_backward(n_in, n_out, packed.data_ptr(), x.data_ptr(), dy.data_ptr(), n,
                                  grad.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    return grad


def mlp_train(n_in: int, n_out: int, params, adam_m, adam_v, adam_t0: int, x16, z16,
              cfg: TrainConfig, stream=None):
    """cfg.updates_per_step Adam steps in place on params / adam_m / adam_v.
    Returns (packed network, per-update losses)."""
    torch = _torch()
    packed = torch.empty(int(lib.srmdp_mlp_packed_bytes()), dtype=torch.uint8, device=params.device)
    loss = torch.empty(cfg.updates_per_step, dtype=torch.float32, device=params.device)
    c = cfg.c()
    nws = int(lib.srmdp_mlp_train_workspace_bytes(n_in, n_out, ctypes.byref(c)))
    ws = torch.empty(max(nws, 256), dtype=torch.uint8, device=params.device)
    _check(lib.srmdp_mlp_train(n_in, n_out, params.data_ptr(), adam_m.data_ptr(), adam_v.data_ptr(),
                               adam_t0, x16.data_ptr(), z16.data_ptr(), x16.shape[0],
                               ctypes.byref(c), packed.data_ptr(), loss.data_ptr(), ws.data_ptr(), nws,
                               _stream_ptr(stream)))
    return packed, loss


def tune_lanes(problem: Problem, grid: Grid, opts: Options, table=None, workspace=None, stream=None):
    """Autotuned lanes per stratum and the time per launch of each candidate
    (8, 16, 32, 64, 128, 256; -1 = not tried).  Overwrites one table row."""
    if table is None:
        table = alloc_table(problem, grid, opts)
    if workspace is None:
        workspace = alloc_workspace(problem, grid, opts, device=table.device)
    lanes = ctypes.c_int32(0)
    ms = (ctypes.c_float * 6)()
    _check(lib.srmdp_tune_lanes(problem.c(), grid.c(), opts.c(), table.data_ptr(), workspace.data_ptr(),
                                workspace.numel(), ctypes.byref(lanes),
                                ctypes.cast(ms, ctypes.POINTER(ctypes.c_float)), _stream_ptr(stream)))
    return int(lanes.value), [float(v) for v in ms]


def _arrays(problems, grids, opts):
    n = len(problems)
    Pa = (_Problem * n)(*[p.c() for p in problems])
    Ga = (_Grid * n)(*[g.c() for g in grids])
    Oa = (_Options * n)(*[o.c() for o in opts])
    return n, Pa, Ga, Oa


def workspace_bytes_batch(problems, grids, opts) -> int:
    n, Pa, Ga, Oa = _arrays(problems, grids, opts)
    v = int(lib.srmdp_workspace_bytes_batch(n, Pa, Ga, Oa))
    if v == 0:
        raise SrmdpError(E_INVALID, lib.srmdp_last_error().decode())
    return v


def solve_batch(problems, grids, opts, tables=None, workspace=None, stream=None, stats: bool = True):
    """Ragged batch of instances in one launch per global backward step.
    Returns (list of tables, list of stats dicts or None)."""
    torch = _torch()
    if tables is None:
        tables = [alloc_table(p, g, o) for p, g, o in zip(problems, grids, opts)]
    n, Pa, Ga, Oa = _arrays(problems, grids, opts)
    if workspace is None:
        workspace = torch.empty(int(lib.srmdp_workspace_bytes_batch(n, Pa, Ga, Oa)) or 1, dtype=torch.uint8,
                                device="cuda")
    ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() for t in tables])
    st = (_Stats * n)()
    _check(lib.srmdp_solve_batch(n, Pa, Ga, Oa, ptrs, workspace.data_ptr(), workspace.numel(),
                                 st if stats else None, _stream_ptr(stream)))
    out = None
    if stats:
        out = [{"singular_cubes": int(x.singular_cubes), "path_steps": int(x.path_steps),
                "ms_total": float(x.ms_total), "step_launches": int(x.step_launches),
                "lanes_per_cube": int(x.lanes_per_cube)} for x in st]
    return tables, out


def release_graphs() -> None:
    lib.srmdp_release_graphs()
