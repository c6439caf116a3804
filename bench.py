#!/usr/bin/env python3
"""Benchmark of the SRMDP backward sweep on one MI355X.

One benchmark step = one full backward sweep (every backward step i = N-1..0
of Algorithm SRMDP: stratified sampling, Euler paths, responses with table
look-ups, z and y regressions, table writes) of the headline workload:
logistic BSDE, d = q = 8, [-3, 3]^8 in 4^8 = 65536 strata, M = 64, N = 50,
LP1, binary32 paths with binary64 Gram sums and solves.  Inputs are synthetic
(the problem is analytic); nothing is read from disk.

Prints one JSON line:
  value        path-steps per second of the whole sweep (K M N(N+1)/2 per sweep)
  roofline     ALU roofline of the sweep-step kernel: algorithmic lane operations
               per launch / average launch time (HIP events around the step
               kernels, on the stream they run on) against the VALU issue peak
  cpu_baseline the FP64 oracle on a bounded sample of the same workload
  ragged_batch the 64-instance ragged batch of d = 2 cos problems in one launch
               per global step, against the same instances solved one by one
  error_matched the full-sweep wall time of the plain estimator and of the
               learned control variate (online training included) at several M,
               with the error of y(0, x0) over seeds (statistical: against the
               scheme's own large-M value; total: against the exact value),
               and the control variate's speed-up at equal statistical error
  cv_equal_M   the d = 4 logistic workload at M = 32: plain against the online
               control variate, same draws; errors of the fitted y and z against
               the closed form and their variance across seeds
  paper_tables the paper's own workloads (rows of its Tables LP0d4 .. LP1d15_19):
               sweep time and the error indicators of eq. (mse), beside the
               values and GPU seconds the paper prints
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

_ROOT = os.path.dirname(os.path.abspath(__file__))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

import workloads as W  # noqa: E402

# MI355X: 256 CUs x 4 SIMDs x 16 lanes per clock x 2.4 GHz = 39.3e12 VALU lane-ops/s;
# FP32 vector 157.3 TFLOP/s (packed FMA).
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
FP32_PEAK_FLOPS = 157.3e12

# per block and lane: 10 rounds of 2 widening 32 x 32 -> 64-bit products and 2
# three-input XORs (4 two-input XOR operations); the key schedule is the same for
# every lane (scalar work) and is not counted
PHILOX_OPS = 10 * (2 + 4)
UNIFORM_OPS = 4                  # shift, or, convert, scale
BOX_MULLER_OPS = 8               # log, sqrt, sincos (2), 4 multiplies per pair
LOCATE_OPS = 8                   # sub, mul, floor, max, min, convert, index fma, xi fma
# equal-probability cells: C F(x) (multiply, exp and its scaling, add, reciprocal,
# multiply), floor, clamp, the index of the cell median in the sampler's table,
# xi = mu (x - median) (subtract, multiply), convert, index fma
LOCATE_OPS_EP = 13

# Bytes beyond L2 per launch of the sweep-step kernel of the default workload, from
# FETCH_SIZE / WRITE_SIZE counter passes scaled by a plain copy's readings (fetch 2.0,
# write 1.0), keyed by a hash of the sources the kernel is compiled from.  A kernel
# built from other sources reports null until it is profiled again.
KERNEL_SOURCES = ("srmdp_kernels.hip", "srmdp_sweep.hpp", "srmdp_device.hpp", "srmdp_internal.hpp",
                  "srmdp_mlp.hpp")
MEASURED_TRAFFIC = {
    "c7abe51ceeecf23e": {"bytes": 4.692e+09,
                         "profile": "profiles/sweep_step_kernel_logistic_d8_K65536_M64_N50.md"},
}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(_ROOT, "paper_2407_21085_amd", "csrc")
    for name in sorted(KERNEL_SOURCES):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_ops(cfg: dict, lookup_terms: int):
    """Lane operations the method needs (lower bound, before compiler overhead).

    Per path-step (d = q here): ceil(q/4) Philox blocks and their 4 uniforms,
    q/2 Box-Muller pairs, q scalings of dW, d Euler adds, d cell locations,
    lookup_terms * d FMAs of the LP evaluations + 2 for truncation, 3 for the
    driver.  Per sample: ceil(d/4) Philox blocks, d uniforms and inverse CDFs
    (2 logs + 6 ops), and the binary64 Gram/right-hand-side products
    nb(nb+1)/2 + q nb + nb plus the y completion q nb + 5.
    """
    d = q = cfg["d"]
    nb = d + 1 if cfg["basis"] == "LP1" else 1
    blocks = math.ceil(q / 4)
    locate = LOCATE_OPS_EP if cfg.get("grid_kind", 0) else LOCATE_OPS
    per_step = (blocks * (PHILOX_OPS + 4 * UNIFORM_OPS) + (q // 2 + q % 2) * BOX_MULLER_OPS
                + q + d + d * locate + lookup_terms * d + 2 + 3)
    per_sample = (math.ceil(d / 4) * PHILOX_OPS + d * (UNIFORM_OPS + 8)
                  + nb * (nb + 1) // 2 + q * nb + nb + q * nb + 5)
    flops_step = 2 * q + d + d * 6 + lookup_terms * 2 * d + 4 + (q // 2) * 6
    return per_step, per_sample, flops_step


def _omp_threads() -> int:
    import oracle as O
    return int(O.max_threads())


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg: dict, seconds: float, full: bool = False) -> dict:
    """The FP64 oracle as it stands.  `value`: the first backward steps of the
    headline workload (steps N-1, N-2, ... until about `seconds` of CPU work,
    all OpenMP threads).  Beside it, whole oracle sweeps of the small
    workloads: cfg1 on all threads and on one, cfg2 and cfg4 on all threads,
    and with `full` cfg2 on one thread (about a minute)."""
    import numpy as np

    import oracle as O
    O.build(force=False)
    sys.path.insert(0, os.path.join(_ROOT, "tests"))
    from sides import oracle_problem
    P = oracle_problem(cfg)
    table = np.zeros(P.table_shape())
    done, t_total, i = 0, 0.0, cfg["N"] - 1
    while i >= 0:
        t0 = time.perf_counter()
        O.solve(P, table=table, i_hi=i, i_lo=i)
        t_total += time.perf_counter() - t0
        done += W.path_steps(cfg, i_hi=i, i_lo=i)
        i -= 1
        if t_total > seconds:
            break
    threads = _omp_threads()
    sweeps = []
    runs = [("cfg1", 0), ("cfg1", 1), ("cfg2", 0), ("cfg4", 0)] + ([("cfg2", 1)] if full else [])
    for name, nthr in runs:
        c = W.config(name)
        Pc = oracle_problem(c)
        t0 = time.perf_counter()
        O.solve(Pc, threads=nthr or threads)   # the count is sticky: always pass it
        dt = time.perf_counter() - t0
        sweeps.append({"workload": c["name"], "threads": nthr or threads, "sweep_s": dt,
                       "path_steps_per_s": W.path_steps(c) / dt})
    return {"value": done / t_total, "unit": "path-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{cfg['name']}: backward steps {cfg['N'] - 1}..{i + 1} "
                      f"({done} FP64 path-steps in {t_total:.1f} s)",
            "host_cpu": _cpu_model(), "host_threads": os.cpu_count(),
            "full_sweeps": sweeps}


def _product_args(S, cfg: dict):
    """The workload as arguments of the HIP library."""
    logistic = cfg["driver"] == "logistic"
    P = S.Problem(d=cfg["d"], N=cfg["N"], T=cfg["T"],
                  driver=S.DRV_LOGISTIC if logistic else S.DRV_LINEAR,
                  terminal=S.G_LOGISTIC if cfg["terminal"] == "logistic" else S.G_COS_SUM,
                  r=cfg.get("r", 0.0), kappa=cfg.get("kappa", 0.0),
                  clamp_y=cfg.get("clamp_y", math.inf))
    G = S.Grid(cfg.get("lo"), cfg.get("hi"), cfg["cells"], cfg["mu"], kind=cfg.get("grid_kind", 0))
    Opt = S.Options(M=cfg["M"], basis=S.LP1 if cfg["basis"] == "LP1" else S.LP0,
                    prec=S.FP32 if cfg["prec"] == "fp32" else S.FP64, seed=cfg["seed"],
                    flags=cfg.get("flags", 0))
    return P, G, Opt


# Learned control variate of the error-matched comparison: the network is
# evaluated every CV_STRIDE steps, trained online with CV_TRAIN after each
# step, and the z response is centred.
CV_STRIDE = 8
CV_TRAIN = dict(updates_per_step=1, batch=16384, lr=1.6e-2)


def _interp_at_error(points, err, value):
    """points[*][value] at statistical error err, interpolated log-log between
    the two measured points that bracket err (None outside their range)."""
    pts = sorted((p["stat_rmse"], p[value]) for p in points)
    for (e0, v0), (e1, v1) in zip(pts, pts[1:]):
        if e0 <= err <= e1 and e0 > 0 and e1 > e0:
            w = math.log(err / e0) / math.log(e1 / e0)
            return math.exp(math.log(v0) + w * (math.log(v1) - math.log(v0)))
    return None


def error_matched(S, cfg: dict, seeds, m_plain, m_cv, m_ref, ref_seeds, root_paths: int, stream,
                  m_small=()) -> dict:
    """Plain estimator at each M in m_plain (the workload's M first) against the
    online control variate at each M in m_cv, over `seeds`: full-sweep time
    (HIP events on the library's stream, training included, mean over seeds)
    and the error of y(0, x0) from the ROOT read-out.  Both sides truncate y at
    C_y = 1, an a-priori bound of this solution (without it the plain
    recursion diverges for some seeds at small M).

    Two errors are reported.  The total error is against the continuous
    solution 0.5.  It contains the discretisation error of the scheme (N time
    steps, LP1 on the strata), which both forms share and no M removes: its
    sign is opposite to that of the small-M noise bias, so the plain total
    error is smallest near M = 64 and then rises to the discretisation error.
    The statistical error, which the number of simulations and the control
    variate act on, is against the scheme's own large-M value y_ref: the mean
    over ref_seeds (seeds of their own) of the plain estimator at m_ref.

    The speed-up at an error eps is T_plain(eps) / T_cv(eps), each time read
    log-log off its own measured (error, time) curve.  It is reported at the
    error of every plain point (the workload's M first, as the target error)
    and at the error of every control-variate point; for the latter the plain
    time is also priced at the plain cost per unit of M at the workload's M,
    and the smaller of the two is kept.  Outside a curve's measured range the
    figure is a bound (lower when the control variate already beats eps at its
    smallest M, or when the plain form needs more than its largest M).

    Each M in m_small (below the curves' range, near the floor M >= d + 1 of
    the LP1 regressions) is reported for both forms beside the curves, not on
    them: there the finite-M bias of the regressions dominates and the error
    is not monotone in M."""
    import torch
    d = cfg["d"]

    def run(M, cv, seed, warm):
        c = dict(cfg, M=M, seed=seed, clamp_y=1.0)
        P, G, Opt = _product_args(S, c)
        if cv:
            Opt.cv, Opt.cv_stride = S.CV_ONLINE, CV_STRIDE
            Opt.flags |= S.F_CV_CENTER_Z
            Opt.cv_train = S.TrainConfig(**CV_TRAIN)
            Opt.cv_params = S.mlp_init(d + 1, d, 1000 + seed, zero_output_layer=True, stream=stream)
        table = S.srmdp.alloc_table(P, G, Opt)
        ws = S.srmdp.alloc_workspace(P, G, Opt)
        ms = 0.0
        for rep in range(2 if warm else 1):  # the first call of a shape warms up
            if cv:
                Opt.cv_params = S.mlp_init(d + 1, d, 1000 + seed, zero_output_layer=True, stream=stream)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(stream):
                ev0.record(stream)
                S.solve(P, G, Opt, table=table, workspace=ws, stream=stream, stats=False)
                ev1.record(stream)
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1)
        y0, _ = S.root(P, G, Opt, table, c["x0"], root_paths, workspace=ws, stream=stream)
        return ms, y0

    def runs(M, cv, seed_list):
        return [run(M, cv, s, n == 0) for n, s in enumerate(seed_list)]

    ref_rows = runs(m_ref, False, ref_seeds)
    ref_y = [y for _, y in ref_rows]
    y_ref = sum(ref_y) / len(ref_y)
    ref_sd = math.sqrt(sum((y - y_ref) ** 2 for y in ref_y) / (len(ref_y) - 1))

    def summary(M, cv):
        rows = runs(M, cv, seeds)
        ys = [y for _, y in rows if math.isfinite(y)]
        out = {"M": M, "ms": sum(t for t, _ in rows) / len(rows), "nonfinite_seeds": len(rows) - len(ys)}
        n = len(ys)
        if n < 2:
            return dict(out, stat_rmse=None, stat_bias=None, sd=None, total_rmse=None)
        mean = sum(ys) / n
        return dict(out, stat_rmse=math.sqrt(sum((y - y_ref) ** 2 for y in ys) / n),
                    stat_bias=mean - y_ref,
                    sd=math.sqrt(sum((y - mean) ** 2 for y in ys) / (n - 1)),
                    total_rmse=math.sqrt(sum((y - 0.5) ** 2 for y in ys) / n))

    plain = [summary(M, False) for M in m_plain]
    cv = [summary(M, True) for M in m_cv]
    small = [{"M": M, "plain": summary(M, False), "cv": summary(M, True)} for M in m_small]
    ms_per_M = plain[0]["ms"] / plain[0]["M"]  # plain cost at the workload, per simulation per stratum
    for c in cv:
        p = next((q for q in plain if q["M"] == c["M"]), None) or summary(c["M"], False)
        c["plain_same_M"] = p
        c["mse_ratio_same_M"] = (p["stat_rmse"] / c["stat_rmse"]) ** 2 if c["stat_rmse"] > 0 else None
        m_eq = _interp_at_error(plain, c["stat_rmse"], "M")
        t_eq = _interp_at_error(plain, c["stat_rmse"], "ms")
        c["plain_M_at_same_error"] = m_eq
        c["speedup_linear"] = ms_per_M * m_eq / c["ms"] if m_eq else None
        c["speedup_measured"] = t_eq / c["ms"] if t_eq else None
        # the smaller of the two: plain cost linear in M from the workload's M, or measured
        c["speedup"] = min(c["speedup_linear"], c["speedup_measured"]) if m_eq and t_eq else None
        if m_eq is None and c["stat_rmse"] < min(q["stat_rmse"] for q in plain):
            # below every plain point: the plain form needs more than its largest M
            top = max(plain, key=lambda q: q["M"])
            c["plain_M_at_same_error_at_least"] = top["M"]
            c["speedup_at_least"] = min(ms_per_M * top["M"], top["ms"]) / c["ms"]
    at_plain = []
    for q in plain:
        t_cv = _interp_at_error(cv, q["stat_rmse"], "ms")
        row = {"plain_M": q["M"], "stat_rmse": q["stat_rmse"], "plain_ms": q["ms"], "cv_ms": t_cv,
               "speedup": q["ms"] / t_cv if t_cv else None}
        if t_cv is None and q["stat_rmse"] > max(c["stat_rmse"] for c in cv):
            # the control variate beats this error at its smallest M
            row["speedup_at_least"] = q["ms"] / min(c["ms"] for c in cv)
        at_plain.append(row)
    scored = [(c.get("speedup") or c.get("speedup_at_least") or 0.0, c) for c in cv]
    best_score, best = max(scored, key=lambda sc: sc[0]) if scored else (0.0, None)
    reached = [r for r in at_plain if (r["speedup"] or 0.0) >= 4.0]
    return {"read_out": f"ROOT y(0,x0), {root_paths} paths", "exact": 0.5, "truncation": "C_y = 1",
            "seeds": list(seeds),
            "reference": {"M": m_ref, "seeds": list(ref_seeds), "y_ref": y_ref,
                          "se": ref_sd / math.sqrt(len(ref_y)), "discretisation_error": y_ref - 0.5},
            "cv_form": {"stride": CV_STRIDE, "centred_z": True, **CV_TRAIN},
            "plain": plain, "cv": cv, "small_M": small,
            "speedup_at_plain_errors": at_plain,
            "at_workload_error": at_plain[0],
            "at_4x_workload_M_error": next((r for r in at_plain if r["plain_M"] == 4 * plain[0]["M"]), None),
            "matched": ({"cv_M": best["M"], "stat_rmse": best["stat_rmse"], "cv_ms": best["ms"],
                         "plain_M_at_same_error": best["plain_M_at_same_error"],
                         "speedup": best_score,
                         "lower_bound": best["plain_M_at_same_error"] is None,
                         "plain_cost": "min(measured, linear in M from the workload's M)"}
                        if best_score > 0 else None),
            "target_reached_from_plain_M": reached[0]["plain_M"] if reached else None,
            "target_speedup": 4.0}


# Forms of the control variate reported at equal M on the d = 4 workload: the
# error-matched comparison's form, and the network evaluated at every step with
# four times the training.
CV_FORMS_EQUAL_M = (
    {"stride": CV_STRIDE, **CV_TRAIN},
    {"stride": 1, "updates_per_step": 4, "batch": 16384, "lr": 1.6e-2},
)


def cv_equal_m(S, cfg: dict, seeds, stream, n_points: int = 4096) -> dict:
    """Plain estimator against the online control variate at the workload's M
    (same draws, same seeds): full-sweep time, and for the fitted y_i, z_i at
    t = 0 and t = T/2 on points drawn uniformly from the central region
    [-1.5, 1.5]^d, the RMS error against the closed form
    u = 1 / (1 + exp(-(t + sum x))), z_l = u (1 - u), and the variance across
    seeds (the mean over the points of the per-point sample variance).  The
    ratios plain / control variate of both are the reported gains."""
    import numpy as np
    import torch
    d = cfg["d"]
    rng = np.random.default_rng(12345)
    pts = rng.uniform(-1.5, 1.5, (n_points, d))
    x = torch.from_numpy(pts).to("cuda")
    torch.cuda.synchronize()  # x is used on `stream`
    steps = (0, cfg["N"] // 2)

    def exact(i):
        t = i * cfg["T"] / cfg["N"]
        u = 1.0 / (1.0 + np.exp(-(t + pts.sum(axis=1))))
        return u, u * (1.0 - u)

    def run(form, seed):
        c = dict(cfg, seed=seed, clamp_y=1.0)
        P, G, Opt = _product_args(S, c)
        if form is not None:
            Opt.cv, Opt.cv_stride = S.CV_ONLINE, form["stride"]
            Opt.flags |= S.F_CV_CENTER_Z
            Opt.cv_train = S.TrainConfig(**{k: v for k, v in form.items() if k != "stride"})
            Opt.cv_params = S.mlp_init(d + 1, d, 1000 + seed, zero_output_layer=True, stream=stream)
        table = S.srmdp.alloc_table(P, G, Opt)
        ws = S.srmdp.alloc_workspace(P, G, Opt)
        times, st = [], None
        for rep in range(2):  # the first call warms up
            if form is not None:
                Opt.cv_params = S.mlp_init(d + 1, d, 1000 + seed, zero_output_layer=True, stream=stream)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(stream):
                ev0.record(stream)
                _, st = S.solve(P, G, Opt, table=table, workspace=ws, stream=stream, stats=rep == 1)
                ev1.record(stream)
            torch.cuda.synchronize()
            times.append(ev0.elapsed_time(ev1))
        fits = []
        for i in steps:
            y, z = S.evaluate(P, G, Opt.basis, Opt.prec, table, i, x, stream=stream)
            torch.cuda.synchronize()
            fits.append((y.cpu().numpy(), z.cpu().numpy()))
        return times[-1], fits, st

    def summary(form):
        rows = [run(form, s) for s in seeds]
        out = {"ms": sum(r[0] for r in rows) / len(rows)}
        for n, i in enumerate(steps):
            u, zu = exact(i)
            ys = np.stack([r[1][n][0] for r in rows])          # [seeds, points]
            zs = np.stack([r[1][n][1] for r in rows])          # [seeds, points, q]
            out[f"i{i}"] = {
                "y_rmse": float(np.sqrt(np.mean((ys - u) ** 2))),
                "z_rmse": float(np.sqrt(np.mean((zs - zu[None, :, None]) ** 2))),
                "y_var": float(np.mean(np.var(ys, axis=0, ddof=1))),
                "z_var": float(np.mean(np.var(zs, axis=0, ddof=1))),
            }
        if form is not None:
            out["form"] = dict(form, centred_z=True)
            out["train_loss_first_last"] = [rows[-1][2]["cv_loss_first"], rows[-1][2]["cv_loss_last"]]
        return out

    plain = summary(None)
    forms = []
    for form in CV_FORMS_EQUAL_M:
        c = summary(form)
        for i in steps:
            p, v = plain[f"i{i}"], c[f"i{i}"]
            v["mse_ratio_y"] = (p["y_rmse"] / v["y_rmse"]) ** 2
            v["mse_ratio_z"] = (p["z_rmse"] / v["z_rmse"]) ** 2
            v["var_ratio_y"] = p["y_var"] / v["y_var"]
            v["var_ratio_z"] = p["z_var"] / v["z_var"]
        forms.append(c)
    return {"workload": cfg["name"], "M": cfg["M"], "seeds": list(seeds), "truncation": "C_y = 1",
            "steps": {f"i{i}": i * cfg["T"] / cfg["N"] for i in steps},
            "points": f"{n_points} uniform on [-1.5, 1.5]^{d}", "plain": plain, "cv": forms}


# Rows of the paper's Tables LP0d4, LP0d6_0, LP0d6_1, LP1d4, LP1d6_1, LP0d11
# and LP1d11 .. LP1d15_19 up to d = 16
# (Section 4: logistic BSDE, X = W, [-6.5, 6.5]^q in #C^q cubes, mu = 1,
# T = 1, binary32): (table, d, basis, N, #C, M, the printed indicators
# (MSE_Y,max, MSE_Y,av, MSE_Z,av) of eq. (mse), the printed GPU seconds on a
# GTX TITAN Black).
PAPER_ROWS = (
    ("LP0d4", 4, "LP0", 20, 17, 400, (-4.337988, -4.698645, -2.302092), 12.39),
    ("LP0d4", 4, "LP0", 50, 28, 2500, (-4.472564, -4.988069, -3.225411), 3070.92),
    ("LP0d6_0", 6, "LP0", 50, 7, 2500, (-3.235130, -3.539011, -2.557686), 874.25),
    ("LP0d6_1", 6, "LP0", 20, 8, 400, (-3.505867, -3.664396, -1.795697), 52.20),
    ("LP1d4", 4, "LP1", 20, 7, 2000, (-4.541253, -5.022405, -2.281332), 7.83),
    ("LP1d4", 4, "LP1", 50, 10, 12500, (-4.574551, -5.143310, -3.228237), 847.83),
    ("LP1d6_1", 6, "LP1", 20, 4, 2800, (-4.075928, -4.231639, -1.791519), 20.50),
    ("LP1d6_1", 6, "LP1", 50, 6, 17500, (-3.809734, -4.529827, -2.689432), 15283.18),
    ("LP0d11", 11, "LP0", 10, 3, 100, (-2.144843, -2.267742, -0.469759), 6.29),
    ("LP0d11", 11, "LP0", 20, 4, 400, (-2.484169, -2.633602, -1.070096), 2108.64),
    ("LP1d11", 11, "LP1", 5, 3, 4000, (-3.269004, -3.403994, -1.975300), 290.56),
    ("LP1d12", 12, "LP1", 5, 3, 4000, (-3.214096, -3.272644, -1.821935), 1196.28),
    ("LP1d13", 13, "LP1", 5, 2, 4000, (-3.022855, -3.158471, -1.649632), 16.58),
    ("LP1d14", 14, "LP1", 5, 2, 4000, (-3.029663, -3.105833, -1.558935), 50.62),
    ("LP1d15_19", 15, "LP1", 5, 2, 5000, (-2.981181, -3.106590, -1.574532), 139.60),
    ("LP1d15_19", 16, "LP1", 5, 2, 6000, (-2.795353, -2.959375, -1.588716), 429.53),
    ("LP1d15_19", 17, "LP1", 5, 2, 5000, (-2.772595, -2.936549, -1.371146), 793.61),
    ("LP1d15_19", 18, "LP1", 5, 2, 4000, (-2.845755, -2.918057, -1.114600), 1589.30),
    ("LP1d15_19", 19, "LP1", 5, 2, 3200, (-2.726427, -2.851617, -0.839849), 4370.31),
)


def paper_tables(S, stream, rows=PAPER_ROWS, points: int = 1000) -> list:
    """The paper's own workloads at their sizes: one binary32 sweep each
    (HIP events on the library's stream; a warm-up sweep first for the small
    ones), and the error indicators of eq. (mse) from 10^3 test points per
    time step drawn from the unrestricted nu (product logistic, mu = 1),
    against y_i = w / (1 + w), z_i = w / (1 + w)^2 with w = exp(t_i + sum x)."""
    import numpy as np
    import torch
    out = []
    for name, d, basis, N, C, M, printed, paper_s in rows:
        cfg = dict(name=f"{name} N={N}", d=d, N=N, T=1.0, lo=[-6.5] * d, hi=[6.5] * d, cells=[C] * d, mu=1.0,
                   M=M, basis=basis, prec="fp32", driver="logistic", terminal="logistic", seed=1)
        P, G, Opt = _product_args(S, cfg)
        table = S.srmdp.alloc_table(P, G, Opt)
        ws = S.srmdp.alloc_workspace(P, G, Opt)
        steps = W.path_steps(cfg)
        reps = 2 if steps < 2e10 else 1
        for _ in range(reps):
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(stream):
                ev0.record(stream)
                _, st = S.solve(P, G, Opt, table=table, workspace=ws, stream=stream)
                ev1.record(stream)
            torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1)
        rng = np.random.default_rng(2024)
        ey, ez = [], []
        for i in range(N):
            u = rng.random((points, d))
            x = np.log(u / (1.0 - u))
            y, z = S.evaluate(P, G, Opt.basis, Opt.prec, table, i, torch.from_numpy(x).cuda(), stream=stream)
            torch.cuda.synchronize()
            w = np.exp(i / N + x.sum(axis=1))
            ey.append(float(np.mean((y.cpu().numpy() - w / (1 + w)) ** 2)))
            ez.append(float(np.mean(((z.cpu().numpy() - (w / (1 + w) ** 2)[:, None]) ** 2).sum(axis=1))))
        mse = (math.log(max(ey)), math.log(sum(ey) / N), math.log(sum(ez) / N))
        out.append({"table": name, "d": d, "basis": basis, "N": N, "cells": C, "K": C ** d, "M": M,
                    "path_steps": steps, "sweep_s": ms / 1e3, "path_steps_per_s": steps / (ms / 1e3),
                    "launches": st["step_launches"], "lanes_per_cube": st["lanes_per_cube"],
                    "mse": [round(v, 4) for v in mse], "paper_mse": list(printed),
                    "paper_gpu_s": paper_s, "paper_gpu": "GTX TITAN Black (context, not the target)"})
        del table, ws
        torch.cuda.empty_cache()
    return out


def ragged_batch(S, stream) -> dict:
    """The ragged batch workload (64 d = 2 cos instances, K 16^2..64^2,
    M 64..1024, N 10..50, binary32): one batched sweep (one launch per global
    step), with heuristic and with autotuned lanes, against the 64 sweeps one
    after the other; HIP events on the library's stream, after a warm-up."""
    import torch
    cfgs = W.ragged_batch()
    args = [_product_args(S, c) for c in cfgs]
    P = [a[0] for a in args]
    G = [a[1] for a in args]
    O = [a[2] for a in args]
    tables = [S.srmdp.alloc_table(p, g, o) for p, g, o in args]
    ws = torch.empty(S.workspace_bytes_batch(P, G, O), dtype=torch.uint8, device="cuda")
    wss = [S.srmdp.alloc_workspace(p, g, o) for p, g, o in args]

    def timed(fn):
        with torch.cuda.stream(stream):
            fn()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            fn()
            ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1)

    batch_ms = timed(lambda: S.solve_batch(P, G, O, tables=tables, workspace=ws, stream=stream, stats=False))
    single_ms = timed(lambda: [S.solve(p, g, o, table=t, workspace=w, stream=stream, stats=False)
                               for (p, g, o), t, w in zip(args, tables, wss)])
    for o in O:
        o.flags |= S.F_AUTOTUNE
    _, st = S.solve_batch(P, G, O, tables=tables, workspace=ws, stream=stream)  # tunes once per shape
    tuned_ms = timed(lambda: S.solve_batch(P, G, O, tables=tables, workspace=ws, stream=stream, stats=False))
    steps = sum(W.path_steps(c) for c in cfgs)
    return {"instances": len(cfgs), "path_steps": steps, "batch_ms": batch_ms,
            "batch_ms_autotuned": tuned_ms, "one_by_one_ms": single_ms,
            "path_steps_per_s": steps / (min(batch_ms, tuned_ms) / 1e3),
            "autotuned_lanes": sorted({s["lanes_per_cube"] for s in st})}


def equal_probability(S, cfg, stream, steps: int, root_paths: int) -> dict:
    """The workload on equal-probability cells (the same cells per dimension,
    cut at the logistic quantiles: every cube of probability 1/K, the outer
    ones unbounded), and for reference on its equal-size cells, both with the
    clouds in LDS: ms per sweep from HIP events on the library's stream after a
    warm-up, path-steps/s, the ALU roofline fraction of each kernel (the longer
    cell location of equal-probability cells counted), and y(0, x0) from the
    ROOT read-out.

    Both runs truncate y at C_y = 1 (eq. (TL); the logistic solution lies in
    (0, 1)): on the unbounded outer cells the few far samples steer the LP1
    slopes, and without truncation the fitted values grow step after step
    until they overflow (in binary64 as in binary32)."""
    import torch
    out = {}
    lookup_terms = 2 if (cfg["driver"] == "logistic" or cfg.get("kappa", 0.0)) else 1
    for key, c, kernel in (("equal_probability", dict(cfg, lo=None, hi=None, grid_kind=1, clamp_y=1.0),
                            "sweep_step_ep_kernel"),
                           ("equal_size", dict(cfg, clamp_y=1.0), "sweep_step_kernel")):
        P, G, Opt = _product_args(S, c)
        table = S.srmdp.alloc_table(P, G, Opt)
        ws = S.srmdp.alloc_workspace(P, G, Opt)
        with torch.cuda.stream(stream):
            S.solve(P, G, Opt, table=table, workspace=ws, stream=stream, stats=False)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            st = [S.solve(P, G, Opt, table=table, workspace=ws, stream=stream, stats=True)[1]
                  for _ in range(steps)]
            ev1.record(stream)
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        ms_steps = sum(x["ms_steps"] for x in st) / steps
        launches = st[0]["step_launches"]
        ops_step, ops_sample, _ = algorithmic_ops(c, lookup_terms)
        K = int(math.prod(c["cells"]))
        ops = W.path_steps(c) * ops_step + K * c["M"] * c["N"] * ops_sample
        y0, _ = S.root(P, G, Opt, table, c["x0"], root_paths, workspace=ws)
        out[key] = {"ms_per_sweep": ms, "path_steps_per_s": W.path_steps(c) / (ms / 1e3),
                    "launches_per_sweep": launches, "avg_launch_ms": ms_steps / launches,
                    "roofline_frac": ops / (ms_steps / 1e3) / VALU_PEAK_OPS,
                    "ops_per_path_step": ops_step, "kernel": kernel, "clamp_y": c["clamp_y"],
                    "y0_root": y0}
        del table, ws
        torch.cuda.empty_cache()
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed full sweeps")
    ap.add_argument("--warmup", type=int, default=2, help="untimed full sweeps")
    ap.add_argument("--workload", default="cfg5", choices=sorted(W.CONFIGS))
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle's cfg2 sweep on one thread (about a minute)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--root-paths", type=int, default=1 << 20)
    ap.add_argument("--no-error-matched", action="store_true",
                    help="skip the plain vs control-variate comparison at matched error")
    ap.add_argument("--em-seeds", type=int, default=32)
    ap.add_argument("--no-cv-equal-m", action="store_true",
                    help="skip the plain vs control-variate comparison at equal M on the d = 4 workload")
    ap.add_argument("--no-paper-tables", action="store_true",
                    help="skip the paper's own workloads (Tables LP0d4 .. LP1d15_19)")
    ap.add_argument("--paper-dims", default="",
                    help="comma-separated dimensions d: run only the paper-table rows of these d (profiling)")
    ap.add_argument("--no-equal-prob", action="store_true",
                    help="skip the workload on equal-probability cells")
    ap.add_argument("--no-ragged-batch", action="store_true",
                    help="skip the 64-instance ragged batch measurement")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run 10 plain device-to-device copies of this many bytes "
                         "(calibrates the HBM byte counters of the profiler)")
    args = ap.parse_args()
    if args.copy_bytes:
        import torch
        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "copies": 10}), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): it measures one GPU's share of the "
              "sweep; sharding the strata over several GPUs is a design, not a measured path.", file=sys.stderr)
        return 2

    import torch

    import paper_2407_21085_amd as S
    from paper_2407_21085_amd import build as _build

    _build.ensure_built(verbose=False)   # compiles only when nothing current is built
    t_start = time.perf_counter()
    cfg = W.config(args.workload)
    P, G, Opt = _product_args(S, cfg)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream()
    table = S.srmdp.alloc_table(P, G, Opt)
    ws = S.srmdp.alloc_workspace(P, G, Opt)
    steps_per_sweep = W.path_steps(cfg)

    def sweep():
        return S.solve(P, G, Opt, table=table, workspace=ws, stream=stream, stats=True)[1]

    with torch.cuda.stream(stream):
        for _ in range(args.warmup):
            sweep()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        stats = [sweep() for _ in range(args.steps)]
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    ms_sweep = ev0.elapsed_time(ev1) / args.steps
    ms_steps = sum(s["ms_steps"] for s in stats) / args.steps
    launches = stats[0]["step_launches"]
    value = steps_per_sweep / (ms_sweep / 1e3)

    lookup_terms = 2 if (cfg["driver"] == "logistic" or cfg.get("kappa", 0.0)) else 1
    ops_step, ops_sample, flops_step = algorithmic_ops(cfg, lookup_terms)
    K = int(math.prod(cfg["cells"]))
    samples = K * cfg["M"] * cfg["N"]
    ops_sweep = steps_per_sweep * ops_step + samples * ops_sample
    avg_launch_s = ms_steps / launches / 1e3
    achieved = ops_sweep / launches / avg_launch_s

    traffic = MEASURED_TRAFFIC.get(kernel_source_hash()) if cfg["name"] == W.config("cfg5")["name"] else None

    y0_root, z0_root = S.root(P, G, Opt, table, cfg["x0"], args.root_paths, workspace=ws)
    x0 = torch.tensor([cfg["x0"]], dtype=torch.float64, device=dev)
    y0_tab, _ = S.evaluate(P, G, Opt.basis, Opt.prec, table, 0, x0)

    out = {
        "metric": "paths·steps/s + full-sweep time at fixed y(0,x0) error, plain vs control-variate",
        "value": value,
        "unit": "path-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_sweep,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic (analytic logistic BSDE, seeded Philox4x32-10 draws)",
        "config": {"workload": cfg["name"], "d": cfg["d"], "K": K, "M": cfg["M"],
                   "N": cfg["N"], "basis": cfg["basis"], "precision": "fp32 paths, fp64 solves",
                   "form": "plain", "parallelism": "1 GPU"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "Tlane-op/s", "frac": achieved / VALU_PEAK_OPS,
                     "traffic": traffic["bytes"] if traffic else None,
                     "traffic_unit": "bytes beyond L2 per launch",
                     "traffic_profile": traffic["profile"] if traffic else None,
                     "kernel": "sweep_step_kernel", "avg_launch_ms": avg_launch_s * 1e3,
                     "launches_per_sweep": launches, "ops_per_path_step": ops_step,
                     "ops_per_sample": ops_sample,
                     "fp32_flop_frac": steps_per_sweep * flops_step / (ms_steps / 1e3)
                     / FP32_PEAK_FLOPS},
        "sweep_ms_kernels_only": ms_steps,
        "wall_s_timed": wall,
        "y0_root": y0_root,
        "y0_table": float(y0_tab.cpu()[0]),
        "y0_exact_continuous": 0.5 if cfg["terminal"] == "logistic" else None,
        "lanes_per_cube": stats[0]["lanes_per_cube"],
    }
    def progress(section):
        # one line per finished section on stderr (the JSON result is the only stdout line)
        print(f"[bench] {section} done after {time.perf_counter() - t_start:.0f} s", file=sys.stderr, flush=True)

    progress("headline sweep")
    if not args.no_equal_prob:
        out["equal_probability"] = equal_probability(S, cfg, stream, args.steps, args.root_paths)
        progress("equal-probability cells")
    if not args.no_ragged_batch:
        out["ragged_batch"] = ragged_batch(S, stream)
        progress("ragged batch")
    if not args.no_paper_tables:
        dims = {int(v) for v in args.paper_dims.split(",") if v.strip()}
        rows = tuple(r for r in PAPER_ROWS if not dims or r[1] in dims)
        out["paper_tables"] = paper_tables(S, stream, rows)
        progress("paper tables")
    if not args.no_error_matched and cfg["driver"] == "logistic":
        M = cfg["M"]
        out["error_matched"] = error_matched(S, cfg, range(1, args.em_seeds + 1), [M, 2 * M, 4 * M, 8 * M],
                                             [M // 2, M, 2 * M], 8 * M, range(1001, 1001 + 2 * args.em_seeds),
                                             1 << 20, stream, m_small=[M // 4])
        progress("error-matched comparison")
    if not args.no_cv_equal_m:
        out["cv_equal_M"] = cv_equal_m(S, W.config("cfg4"), range(1, 5), stream)
        progress("equal-M comparison")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds, full=args.cpu_full)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
