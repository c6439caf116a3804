"""MI355X (gfx950) implementation of the backward dynamic-programming sweep of
the stratified regression Monte-Carlo scheme (SRMDP) for BSDEs and semilinear
PDEs, arXiv 2407.21085.

The computation lives in libsrmdp.so (HIP kernels behind the C ABI declared in
include/srmdp.h); `srmdp` is its thin ctypes binding.
"""
from . import srmdp  # noqa: F401  (loads libsrmdp.so; raises ImportError if it is not built)
from .srmdp import (CV_FROZEN, CV_NONE, CV_ONLINE, DRV_LINEAR, DRV_LOGISTIC,  # noqa: F401
                    F_AUTOTUNE, F_CHECK_FINITE, F_CV_CENTER_Z, F_GLOBAL_ROWS, F_GRAPH, FP32, FP64,
                    GRID_EQUAL_PROB, GRID_EQUAL_SIZE,
                    G_COS_SUM, G_LOGISTIC, LP0, LP1, Grid,
                    Options, Problem, SrmdpError, TrainConfig, cv_pairs, draw, evaluate,
                    mlp_backward, mlp_forward, mlp_init, mlp_pack, mlp_param_count, mlp_train,
                    release_graphs, root, solve, solve_batch, table_elems, tune_lanes,
                    workspace_bytes, workspace_bytes_batch)
