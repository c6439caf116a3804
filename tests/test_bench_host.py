"""Host-side pieces of bench.py that need no GPU: the algorithmic operation
count of the headline workload, the matched-error interpolation, and the
--gpus guard."""
import math
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench as B  # noqa: E402
import workloads as W  # noqa: E402


def test_algorithmic_ops_of_the_headline_workload():
    """d = q = 8, LP1, two look-up terms (logistic driver): 285 lane operations per
    path-step and 419 per sample, the counts the roofline is quoted on."""
    per_step, per_sample, _ = B.algorithmic_ops(W.config("cfg5"), 2)
    assert per_step == 285
    assert per_sample == 419
    # equal-probability cells: 13 operations per cell location instead of 8
    per_step_ep, per_sample_ep, _ = B.algorithmic_ops(dict(W.config("cfg5"), grid_kind=1), 2)
    assert per_step_ep == 285 + 8 * 5
    assert per_sample_ep == 419


PLAIN = [{"M": 64, "ms": 60.0, "stat_rmse": 0.008}, {"M": 128, "ms": 140.0, "stat_rmse": 0.004},
         {"M": 256, "ms": 350.0, "stat_rmse": 0.003}]


def test_interpolation_at_error_is_log_log_between_brackets():
    # the end points are returned exactly
    assert B._interp_at_error(PLAIN, 0.008, "M") == pytest.approx(64)
    assert B._interp_at_error(PLAIN, 0.003, "ms") == pytest.approx(350.0)
    # half-way in log error between 0.004 and 0.008 is half-way in log M
    e = math.sqrt(0.004 * 0.008)
    assert B._interp_at_error(PLAIN, e, "M") == pytest.approx(math.sqrt(64 * 128))
    # outside the measured range: no value
    assert B._interp_at_error(PLAIN, 0.002, "M") is None
    assert B._interp_at_error(PLAIN, 0.01, "M") is None


def test_interpolation_ignores_the_order_of_the_points():
    assert B._interp_at_error(PLAIN[::-1], 0.0035, "M") == pytest.approx(B._interp_at_error(PLAIN, 0.0035, "M"))


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
