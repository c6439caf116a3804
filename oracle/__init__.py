"""FP64 CPU oracle of the SRMDP backward sweep (arXiv 2407.21085, Algorithm SRMDP).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark import this package.  It shares no code with the
HIP library: the C source next to this file is a separate, plain
implementation of the paper's algorithm in binary64.

The Python side only marshals arguments (numpy arrays) into the C oracle and
holds the numerical helpers the pins need.
"""
from __future__ import annotations

import contextlib
import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "srmdp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libsrmdp_oracle.so")

LP0, LP1 = 0, 1
DRV_LINEAR, DRV_LOGISTIC = 0, 1
G_COS_SUM, G_LOGISTIC = 0, 1
GRID_EQUAL_SIZE, GRID_EQUAL_PROB = 0, 1


def compile_source(src: str, out: str, extra_flags=()) -> str:
    """gcc -O2, no fast-math, no contraction, OpenMP over strata (extra_flags:
    an instrumented build, for instance)."""
    tmp = out + ".tmp"
    cmd = (["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared"] +
           list(extra_flags) + ["-I", _HERE, src, "-o", tmp, "-lm"])
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compiles the oracle library next to its source."""
    if force or not os.path.exists(_LIB_PATH):
        compile_source(_SRC, _LIB_PATH)
    return _LIB_PATH


@contextlib.contextmanager
def using_library(path: str):
    """Temporarily routes every oracle call to another build of the oracle
    (used by the tests that plant a mistake in a copy of the source)."""
    global _lib
    saved = _lib
    _lib = None
    _bind(ctypes.CDLL(path))
    try:
        yield
    finally:
        _lib = saved


class _Model(ctypes.Structure):
    _fields_ = [("b", ctypes.c_void_p), ("sigma_dw", ctypes.c_void_p), ("f", ctypes.c_void_p),
                ("g", ctypes.c_void_p), ("params", ctypes.POINTER(ctypes.c_double)),
                ("lip_y", ctypes.c_double), ("lip_z", ctypes.c_double)]


class _Problem(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32), ("q", ctypes.c_int32),
        ("T", ctypes.c_double), ("N", ctypes.c_int32),
        ("b", ctypes.POINTER(ctypes.c_double)), ("sigma", ctypes.POINTER(ctypes.c_double)),
        ("driver", ctypes.c_int32), ("terminal", ctypes.c_int32),
        ("r", ctypes.c_double), ("kappa", ctypes.c_double),
        ("clamp_y", ctypes.c_double), ("clamp_z", ctypes.c_double),
        ("lo", ctypes.POINTER(ctypes.c_double)), ("hi", ctypes.POINTER(ctypes.c_double)),
        ("cells", ctypes.POINTER(ctypes.c_int32)), ("mu", ctypes.c_double),
        ("M", ctypes.c_int32), ("basis", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("inst", ctypes.c_uint32),
        ("cv_params", ctypes.POINTER(ctypes.c_double)), ("cv_hidden", ctypes.c_int32),
        ("cv_bf16", ctypes.c_int32),
        ("face_flags", ctypes.c_void_p), ("face_eps", ctypes.c_double),
        ("cv_stride", ctypes.c_int32), ("z_center", ctypes.c_int32),
        ("b_lin", ctypes.POINTER(ctypes.c_double)),
        ("grid_kind", ctypes.c_int32),
        ("sigma_lin", ctypes.POINTER(ctypes.c_double)),
        ("flip_bound", ctypes.POINTER(ctypes.c_double)),
        ("face_flip", ctypes.c_int32),
        ("debug_singular", ctypes.c_int32),
        ("debug_singular_step", ctypes.c_int32),
        ("debug_singular_stratum", ctypes.c_int64),
        ("model", ctypes.POINTER(_Model)),
    ]


_lib = None


def lib():
    if _lib is None:
        # SRMDP_ORACLE_LIBRARY names another build of the oracle (an instrumented one)
        path = os.environ.get("SRMDP_ORACLE_LIBRARY")
        if not path:
            path = _LIB_PATH
            if not os.path.exists(path):
                build(force=True)
        _bind(ctypes.CDLL(path))
    return _lib


def _bind(L):
    global _lib
    dp = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(_Problem)
    L.orc_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
    L.orc_path_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32,
                                    ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int32, dp]
    L.orc_start_point.argtypes = [pp, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32, dp]
    L.orc_path_normals.argtypes = [pp, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_int32, dp]
    L.orc_table_elems.argtypes = [pp]
    L.orc_table_elems.restype = ctypes.c_int64
    L.orc_solve.argtypes = [pp, dp, ctypes.c_int32, ctypes.c_int32,
                            ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]
    L.orc_cloud.argtypes = [pp, dp, ctypes.c_int32, ctypes.c_uint32, dp, dp, dp, dp, dp]
    L.orc_eval.argtypes = [pp, dp, ctypes.c_int32, ctypes.c_int64, dp, dp, dp]
    L.orc_root.argtypes = [pp, dp, dp, ctypes.c_int32, dp, dp]
    L.orc_driver.argtypes = [pp, ctypes.c_double, dp, ctypes.c_double, dp]
    L.orc_driver.restype = ctypes.c_double
    L.orc_terminal.argtypes = [pp, dp]
    L.orc_terminal.restype = ctypes.c_double
    L.orc_max_threads.argtypes = []
    L.orc_max_threads.restype = ctypes.c_int
    L.orc_mlp_param_count.argtypes = [ctypes.c_int32] * 3
    L.orc_mlp_param_count.restype = ctypes.c_int64
    L.orc_mlp_forward.argtypes = [ctypes.c_int32] * 3 + [dp, dp, ctypes.c_int64, dp]
    L.orc_mlp_backward.argtypes = [ctypes.c_int32] * 3 + [dp, dp, dp, ctypes.c_int64, dp]
    L.orc_mlp_forward_bf.argtypes = [ctypes.c_int32] * 3 + [dp, dp, ctypes.c_int64, dp,
                                                            ctypes.c_int32]
    L.orc_mlp_backward_bf.argtypes = [ctypes.c_int32] * 3 + [dp, dp, dp, ctypes.c_int64, dp,
                                                             ctypes.c_int32]
    _lib = L


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


_MODEL_LIBS = {}


@dataclass
class Model:
    """A problem's own coefficients as a small C plugin, compiled with gcc
    (-DMODEL_D=d) and called by the oracle through function pointers.  The
    source defines
        void model_b(double t, const double *x, const double *p, double *out);
        void model_sigma_dw(double t, const double *x, const double *dw, const double *p, double *out);
        double model_f(double t, const double *x, double y, const double *z, const double *p);
        double model_g(const double *x, const double *p);
    lip_y, lip_z bound |df/dy| and |df/dz_l| (used by the face-flip bound only)."""
    source: str
    params: Sequence[float] = ()
    lip_y: float = 0.0
    lip_z: float = 0.0

    def library(self, d: int):
        import hashlib
        import tempfile
        key = hashlib.sha256(f"{d}\n{self.source}".encode()).hexdigest()[:20]
        if key not in _MODEL_LIBS:
            tmp = os.path.join(tempfile.gettempdir(), f"srmdp_oracle_model_{os.getuid()}")
            os.makedirs(tmp, exist_ok=True)
            src = os.path.join(tmp, f"model_{key}.c")
            out = os.path.join(tmp, f"libmodel_{key}.so")
            if not os.path.exists(out):
                with open(src, "w") as f:
                    f.write(self.source)
                subprocess.run(["gcc", "-O2", "-std=c99", "-fno-fast-math", "-ffp-contract=off", "-fPIC",
                                "-shared", f"-DMODEL_D={d}", src, "-o", out + ".tmp", "-lm"], check=True)
                os.replace(out + ".tmp", out)
            _MODEL_LIBS[key] = ctypes.CDLL(out)
        return _MODEL_LIBS[key]


@dataclass
class Problem:
    """Problem data, stratification and simulation settings of one sweep."""
    d: int
    N: int
    lo: Optional[Sequence[float]]   # ignored (may be None) for GRID_EQUAL_PROB
    hi: Optional[Sequence[float]]
    cells: Sequence[int]
    M: int
    T: float = 1.0
    q: Optional[int] = None
    basis: int = LP1
    driver: int = DRV_LINEAR
    terminal: int = G_COS_SUM
    r: float = 0.0
    kappa: float = 0.0
    mu: float = 1.0
    clamp_y: float = math.inf
    clamp_z: float = math.inf
    b: Optional[Sequence[float]] = None
    b_lin: Optional[Sequence[float]] = None   # drift b_l + b_lin_l x_l
    sigma: Optional[Sequence[float]] = None
    seed: int = 1
    inst: int = 0
    cv_params: Optional[np.ndarray] = None
    cv_hidden: int = 0
    cv_bf16: int = 0
    face_flags: Optional[np.ndarray] = None   # uint8 [N, K] diagnostic output
    face_eps: float = 1e-5
    cv_stride: int = 1
    z_center: int = 0
    grid_kind: int = GRID_EQUAL_SIZE
    sigma_lin: Optional[Sequence[float]] = None   # diffusion sigma + diag(sigma_lin) x
    # test diagnostics: per-coefficient bound of a face flip (float64 [N, K, 1+q, nb]
    # output), forced flips, and a Gram matrix zeroed at (step, stratum)
    flip_bound: Optional[np.ndarray] = None
    face_flip: int = 0
    debug_singular: Optional[tuple] = None
    model: Optional[Model] = None   # the problem's own coefficients (C plugin)
    _keep: list = field(default_factory=list, repr=False)

    def __post_init__(self):
        if self.q is None:
            self.q = self.d

    @property
    def K(self) -> int:
        return int(np.prod(np.asarray(self.cells, dtype=np.int64)))

    @property
    def nb(self) -> int:
        return self.d + 1 if self.basis == LP1 else 1

    @property
    def dt(self) -> float:
        return self.T / self.N

    def table_shape(self):
        return (self.N, self.K, 1 + self.q, self.nb)

    def c(self) -> _Problem:
        keep = []

        def arr(v, dtype=np.float64):
            if v is None:
                return None
            a = np.ascontiguousarray(np.asarray(v, dtype=dtype))
            keep.append(a)
            return a

        lo, hi = arr(self.lo), arr(self.hi)
        cells = arr(self.cells, np.int32)
        b, sig, blin, slin = arr(self.b), arr(self.sigma), arr(self.b_lin), arr(self.sigma_lin)
        cvp = arr(self.cv_params)
        s = _Problem()
        s.d, s.q, s.T, s.N = self.d, self.q, self.T, self.N
        s.b = _dp(b) if b is not None else None
        s.sigma = _dp(sig) if sig is not None else None
        s.driver, s.terminal, s.r, s.kappa = self.driver, self.terminal, self.r, self.kappa
        s.clamp_y, s.clamp_z = self.clamp_y, self.clamp_z
        s.lo = _dp(lo) if lo is not None else None
        s.hi = _dp(hi) if hi is not None else None
        s.cells = cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        s.mu, s.M, s.basis = self.mu, self.M, self.basis
        s.seed, s.inst = self.seed, self.inst
        s.cv_params = _dp(cvp) if cvp is not None else None
        s.cv_hidden = self.cv_hidden if cvp is not None else 0
        s.cv_bf16 = self.cv_bf16
        if self.face_flags is not None:
            assert self.face_flags.dtype == np.uint8 and self.face_flags.flags["C_CONTIGUOUS"]
            assert self.face_flags.shape == (self.N, self.K)
            s.face_flags = self.face_flags.ctypes.data
        s.face_eps = self.face_eps
        s.cv_stride = self.cv_stride
        s.z_center = self.z_center
        s.b_lin = _dp(blin) if blin is not None else None
        s.grid_kind = self.grid_kind
        s.sigma_lin = _dp(slin) if slin is not None else None
        if self.flip_bound is not None:
            fb = self.flip_bound
            assert fb.dtype == np.float64 and fb.flags["C_CONTIGUOUS"] and fb.shape == self.table_shape()
            s.flip_bound = _dp(fb)
        s.face_flip = int(self.face_flip)
        if self.debug_singular is not None:
            s.debug_singular = 1
            s.debug_singular_step, s.debug_singular_stratum = (int(v) for v in self.debug_singular)
        if self.model is not None:
            lib_m = self.model.library(self.d)
            prm = arr(list(self.model.params) or [0.0])
            fn = [ctypes.cast(getattr(lib_m, n), ctypes.c_void_p).value
                  for n in ("model_b", "model_sigma_dw", "model_f", "model_g")]
            m = _Model(*fn, _dp(prm), float(self.model.lip_y), float(self.model.lip_z))
            keep += [lib_m, m]
            s.model = ctypes.pointer(m)
        self._keep = keep
        return s


def max_threads() -> int:
    return int(lib().orc_max_threads())


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = (ctypes.c_uint32 * 4)(*ctr)
    k = (ctypes.c_uint32 * 2)(*key)
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def path_uniforms(seed: int, inst: int, i: int, k: int, m: int, n: int) -> np.ndarray:
    u = np.empty(n, dtype=np.float64)
    lib().orc_path_uniforms(seed, inst, i, k, m, n, _dp(u))
    return u


def start_point(P: Problem, i: int, k: int, m: int) -> np.ndarray:
    x = np.empty(P.d, dtype=np.float64)
    rc = lib().orc_start_point(ctypes.byref(P.c()), i, k, m, _dp(x))
    if rc != 0:
        raise ValueError("invalid problem")
    return x


def path_normals(P: Problem, i: int, k: int, m: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().orc_path_normals(ctypes.byref(P.c()), i, k, m, n, _dp(out))
    return out


def solve(P: Problem, table: Optional[np.ndarray] = None, i_hi: Optional[int] = None,
          i_lo: int = 0, threads: int = 0):
    """Algorithm SRMDP for i = i_hi .. i_lo; returns (table[N,K,1+q,nb], singular)."""
    if table is None:
        table = np.zeros(P.table_shape(), dtype=np.float64)
    assert table.shape == P.table_shape() and table.dtype == np.float64
    assert table.flags["C_CONTIGUOUS"]
    if i_hi is None:
        i_hi = P.N - 1
    sing = ctypes.c_int64(0)
    rc = lib().orc_solve(ctypes.byref(P.c()), _dp(table), i_hi, i_lo, ctypes.byref(sing),
                         threads)
    if rc != 0:
        raise ValueError("invalid problem")
    return table, int(sing.value)


def cloud(P: Problem, table: np.ndarray, i: int, k: int):
    """The simulations of stratum k at step i (given fitted rows > i)."""
    M, d, q = P.M, P.d, P.q
    Xi = np.empty((M, d)); dW = np.empty((M, q)); Sp = np.empty(M); y1 = np.empty(M)
    cvi = np.empty(M)
    rc = lib().orc_cloud(ctypes.byref(P.c()), _dp(table), i, k, _dp(Xi), _dp(dW), _dp(Sp),
                         _dp(y1), _dp(cvi))
    if rc != 0:
        raise ValueError("invalid problem")
    return Xi, dW, Sp, y1, cvi


def evaluate(P: Problem, table: np.ndarray, i: int, x: np.ndarray):
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, P.d)
    n = x.shape[0]
    y = np.empty(n); z = np.empty((n, P.q))
    rc = lib().orc_eval(ctypes.byref(P.c()), _dp(table), i, n, _dp(x), _dp(y), _dp(z))
    if rc != 0:
        raise ValueError("invalid problem")
    return y, z


def root(P: Problem, table: np.ndarray, x0: Sequence[float], M_root: int):
    x0 = np.ascontiguousarray(x0, dtype=np.float64)
    y0 = ctypes.c_double(0.0)
    z0 = np.empty(P.q)
    rc = lib().orc_root(ctypes.byref(P.c()), _dp(table), _dp(x0), M_root, ctypes.byref(y0),
                        _dp(z0))
    if rc != 0:
        raise ValueError("invalid problem")
    return float(y0.value), z0


def table_readout(P: Problem, table: np.ndarray, x0: Sequence[float]):
    y, z = evaluate(P, table, 0, np.asarray(x0, dtype=np.float64)[None, :])
    return float(y[0]), z[0]


def driver(P: Problem, t: float, x, y: float, z) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    return float(lib().orc_driver(ctypes.byref(P.c()), t, _dp(x), y, _dp(z)))


def terminal(P: Problem, x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(lib().orc_terminal(ctypes.byref(P.c()), _dp(x)))


def mlp_param_count(n_in: int, H: int, n_out: int) -> int:
    return int(lib().orc_mlp_param_count(n_in, H, n_out))


BF_WEIGHTS, BF_INPUT, BF_HIDDEN, BF_GRADS, BF_PAIR = 1, 2, 4, 8, 16
# the arithmetic of the library's network: bf16 weights, inputs as bf16 pairs,
# bf16 hidden activations and gradient operands
BF_ALL = BF_WEIGHTS | BF_PAIR | BF_HIDDEN | BF_GRADS


def mlp_forward(n_in: int, H: int, n_out: int, params: np.ndarray, x: np.ndarray,
                bf: int = 0) -> np.ndarray:
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, n_in)
    y = np.empty((x.shape[0], n_out))
    lib().orc_mlp_forward_bf(n_in, H, n_out, _dp(params), _dp(x), x.shape[0], _dp(y), bf)
    return y


def mlp_backward(n_in: int, H: int, n_out: int, params: np.ndarray, x: np.ndarray,
                 dy: np.ndarray, bf: int = 0) -> np.ndarray:
    params = np.ascontiguousarray(params, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, n_in)
    dy = np.ascontiguousarray(dy, dtype=np.float64).reshape(-1, n_out)
    g = np.empty(params.size)
    lib().orc_mlp_backward_bf(n_in, H, n_out, _dp(params), _dp(x), _dp(dy), x.shape[0], _dp(g),
                              bf)
    return g
