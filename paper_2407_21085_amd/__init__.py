"""MI355X (gfx950) implementation of the backward dynamic-programming sweep of
the stratified regression Monte-Carlo scheme (SRMDP) for BSDEs and semilinear
PDEs, arXiv 2407.21085.

The computation lives in libsrmdp.so (HIP kernels behind the C ABI declared in
include/srmdp.h); `srmdp` is its thin ctypes binding.
"""
from . import srmdp  # noqa: F401  (loads libsrmdp.so; raises ImportError if it is not built)
from .srmdp import (DRV_LINEAR, DRV_LOGISTIC, F_CHECK_FINITE, F_GRAPH, FP32, FP64, G_COS_SUM,  # noqa: F401
                    G_LOGISTIC, LP0, LP1, Grid, Options, Problem, SrmdpError, draw, evaluate,
                    release_graphs, root, solve, table_elems, workspace_bytes)
