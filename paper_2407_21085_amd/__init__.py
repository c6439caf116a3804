"""MI355X (gfx950) implementation of the backward dynamic-programming sweep of
the stratified regression Monte-Carlo scheme (SRMDP) for BSDEs and semilinear
PDEs, arXiv 2407.21085.

The computation lives in libsrmdp.so (HIP kernels behind the C ABI declared in
include/srmdp.h); `srmdp` is its thin ctypes binding.

The binding is imported lazily, on the first access to one of its names, so
that `paper_2407_21085_amd.build` can be imported (and run) on a tree where
libsrmdp.so does not exist yet.  Accessing any binding name without the
library raises ImportError.
"""
from __future__ import annotations

import importlib

_BINDING_NAMES = frozenset((
    "CV_FROZEN", "CV_NONE", "CV_ONLINE", "DRV_LINEAR", "DRV_LOGISTIC",
    "F_AUTOTUNE", "F_CHECK_FINITE", "F_CV_CENTER_Z", "F_DEBUG_SINGULAR", "F_GLOBAL_ROWS", "F_GRAPH", "FP32", "FP64",
    "GRID_EQUAL_PROB", "GRID_EQUAL_SIZE", "G_COS_SUM", "G_LOGISTIC", "LP0", "LP1", "Grid", "Model",
    "Options", "Problem", "SrmdpError", "TrainConfig", "cv_pairs", "draw", "evaluate", "to_raw_basis",
    "mlp_backward", "mlp_forward", "mlp_init", "mlp_pack", "mlp_param_count", "mlp_train",
    "release_graphs", "root", "solve", "solve_batch", "solve_noalloc", "table_elems", "tune_lanes",
    "workspace_bytes", "workspace_bytes_batch",
))

__all__ = sorted(_BINDING_NAMES) + ["srmdp", "build", "ensure_built"]


def ensure_built(verbose: bool = False) -> str:
    """Builds libsrmdp.so in-tree when it is missing or older than a source.

    Returns the library path.  Compiles nothing when the library is newer
    than every file under csrc/ and include/.
    """
    from . import build as _b
    return _b.ensure_built(verbose=verbose)


def __getattr__(name: str):
    if name == "srmdp":
        return importlib.import_module(".srmdp", __name__)
    if name in _BINDING_NAMES:
        mod = importlib.import_module(".srmdp", __name__)
        return getattr(mod, name)
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")


def __dir__():
    return sorted(set(globals()) | _BINDING_NAMES | {"srmdp", "build"})
