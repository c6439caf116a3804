"""Translates a workload (workloads.py) into the arguments of each side: the
oracle's Problem and the HIP library's (Problem, Grid, Options)."""
import math

import oracle as O

_BASIS = {"LP0": 0, "LP1": 1}
_DRIVER = {"linear": 0, "logistic": 1}
_TERMINAL = {"cos": 0, "logistic": 1}


def oracle_problem(cfg, **kw):
    c = dict(cfg)
    c.update(kw)
    return O.Problem(d=c["d"], N=c["N"], T=c["T"], lo=c.get("lo"), hi=c.get("hi"), cells=c["cells"],
                     M=c["M"], basis=_BASIS[c["basis"]], driver=_DRIVER[c["driver"]],
                     terminal=_TERMINAL[c["terminal"]], r=c.get("r", 0.0),
                     kappa=c.get("kappa", 0.0), mu=c["mu"], seed=c["seed"],
                     inst=c.get("instance", 0), clamp_y=c.get("clamp_y", math.inf),
                     face_flags=c.get("face_flags"), face_eps=c.get("face_eps", 1e-5),
                     clamp_z=c.get("clamp_z", math.inf), b=c.get("b"), sigma=c.get("sigma"),
                     b_lin=c.get("b_lin"), grid_kind=c.get("grid_kind", 0), sigma_lin=c.get("sigma_lin"))


def product_args(cfg, **kw):
    import paper_2407_21085_amd as S
    c = dict(cfg)
    c.update(kw)
    P = S.Problem(d=c["d"], N=c["N"], T=c["T"], driver=_DRIVER[c["driver"]],
                  terminal=_TERMINAL[c["terminal"]], r=c.get("r", 0.0), kappa=c.get("kappa", 0.0),
                  clamp_y=c.get("clamp_y", math.inf), clamp_z=c.get("clamp_z", math.inf),
                  b=c.get("b"), sigma=c.get("sigma"), b_lin=c.get("b_lin"), sigma_lin=c.get("sigma_lin"))
    G = S.Grid(c.get("lo"), c.get("hi"), c["cells"], c["mu"], kind=c.get("grid_kind", 0))
    Opt = S.Options(M=c["M"], basis=_BASIS[c["basis"]], prec=S.FP32 if c["prec"] == "fp32" else S.FP64,
                    seed=c["seed"], instance=c.get("instance", 0), step_hi=c.get("step_hi", -1),
                    step_lo=c.get("step_lo", -1), lanes_per_cube=c.get("lanes", 0),
                    flags=c.get("flags", 0), global_rows_strata=c.get("global_rows_strata", 0))
    return P, G, Opt
