"""Pins of test diagnostics of the oracle (CPU only).

1. The face-flip bound.  A look-up point within eps cell widths of an interior
   cell face may fall in the neighbouring cube when computed in another
   precision.  The oracle bounds, per coefficient, how far such choices can
   move a stratum's fit (each path's response change through the regression's
   leverage G^-1 phi_m, Section 3.1's OLS).  Pinned by brute force: a run in
   which every near-face look-up takes the cube across its face must stay
   within the bound, coefficient by coefficient, and the bound must be of the
   size of the change it bounds (not vacuous).

   The same bound covers the control-variate network's bfloat16 roundings:
   a hidden activation within a few binary32 units of a rounding midpoint may
   round to the other neighbour in another precision; the forced run rounds
   every such activation the other way.

2. The singular-Gram fallback.  A Gram matrix forced to zero at one (step,
   stratum) must give that stratum the LP0 fit, i.e. the empirical means of
   the responses (Section 4.1, explicit LP0 solution), computed here from the
   stratum's cloud, and leave every other stratum bit for bit unchanged.
"""
import math

import numpy as np
import pytest

import oracle as O

CASES = [
    # (name, problem overrides, eps in cell widths)
    ("logistic d=2", dict(d=2, N=6, lo=[-3.0] * 2, hi=[3.0] * 2, cells=[6, 6], M=40, driver=O.DRV_LOGISTIC,
                          terminal=O.G_LOGISTIC), 0.03),
    ("linear kappa d=3 clamps", dict(d=3, N=5, lo=[-2.0] * 3, hi=[2.0] * 3, cells=[3, 4, 3], M=30,
                                     driver=O.DRV_LINEAR, r=0.4, kappa=0.6, clamp_y=0.8, clamp_z=0.5), 0.03),
    ("logistic d=2 centred z", dict(d=2, N=5, lo=[-3.0] * 2, hi=[3.0] * 2, cells=[5, 4], M=40,
                                    driver=O.DRV_LOGISTIC, terminal=O.G_LOGISTIC, z_center=1), 0.03),
    ("linear d=1 lp0", dict(d=1, N=8, lo=[-4.0], hi=[4.0], cells=[16], M=50, basis=O.LP0, driver=O.DRV_LINEAR,
                            r=0.2, kappa=0.5), 0.05),
]


def _problem(kw, **extra):
    base = dict(T=1.0, mu=1.0, seed=7)
    base.update(kw)
    base.update(extra)
    return O.Problem(**base)


@pytest.mark.parametrize("name,kw,eps", CASES, ids=[c[0] for c in CASES])
def test_flip_bound_holds_against_forced_flips(name, kw, eps):
    P0 = _problem(kw)
    table, _ = O.solve(P0)
    K, i = P0.K, 1
    flags = np.zeros((P0.N, K), dtype=np.uint8)
    bound = np.zeros(P0.table_shape())
    Pb = _problem(kw, face_flags=flags, face_eps=eps, flip_bound=bound)
    base = table.copy()
    O.solve(Pb, table=base, i_hi=i, i_lo=i)
    flipped = table.copy()
    O.solve(_problem(kw, face_eps=eps, face_flip=1), table=flipped, i_hi=i, i_lo=i)

    change = np.abs(flipped[i] - base[i])
    b = bound[i]
    assert flags[i].any(), "the case must have near-face look-ups"
    # unflagged strata: no candidate cube, so a zero bound and no change
    assert np.all(b[flags[i] == 0] == 0.0)
    assert np.all(change[flags[i] == 0] == 0.0)
    # every coefficient within its bound (rounding slack of the two solves)
    scale = np.max(np.abs(base[i]))
    assert np.all(change <= b + 1e-12 * scale), np.max(change - b)
    # the bound is of the size of what it bounds on the strata that changed
    moved = change.reshape(K, -1).max(axis=1) > 1e-9 * scale
    assert moved.sum() >= 2
    ratio = change.reshape(K, -1).max(axis=1)[moved] / b.reshape(K, -1).max(axis=1)[moved]
    assert ratio.max() > 0.2, ratio


def test_flip_bound_does_not_change_the_fit():
    """Asking for the bound, the flags or both leaves the table bit for bit
    the same (the diagnostics only read)."""
    kw = CASES[0][1]
    P0 = _problem(kw)
    ref, _ = O.solve(P0)
    flags = np.zeros((P0.N, P0.K), dtype=np.uint8)
    bound = np.zeros(P0.table_shape())
    got, _ = O.solve(_problem(kw, face_flags=flags, face_eps=0.05, flip_bound=bound))
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("basis,driver", [(O.LP1, O.DRV_LOGISTIC), (O.LP1, O.DRV_LINEAR), (O.LP0, O.DRV_LINEAR)])
def test_singular_gram_takes_the_lp0_mean(basis, driver):
    kw = dict(d=2, N=4, lo=[-2.0] * 2, hi=[2.0] * 2, cells=[3, 3], M=25, basis=basis, driver=driver,
              terminal=O.G_LOGISTIC if driver == O.DRV_LOGISTIC else O.G_COS_SUM, r=0.3, kappa=0.4,
              clamp_z=0.9)
    P0 = _problem(kw)
    ref, sing0 = O.solve(P0)
    assert sing0 == 0
    i, k = 1, 4
    Ps = _problem(kw, debug_singular=(i, k))
    table = ref.copy()
    _, sing = O.solve(Ps, table=table, i_hi=i, i_lo=i)
    assert sing == 1
    others = np.ones(P0.K, dtype=bool)
    others[k] = False
    np.testing.assert_array_equal(table[i][others], ref[i][others])
    np.testing.assert_array_equal(table[i + 1:], ref[i + 1:])
    # explicit LP0 solution: the empirical means of the responses of the cloud
    X, dW, Sp, y1, cvi = O.cloud(P0, ref, i, k)
    dt = P0.dt
    rec = table[i, k]
    for l in range(P0.q):
        assert rec[1 + l, 0] == pytest.approx(np.mean(Sp * dW[:, l] / dt), rel=1e-12, abs=1e-14)
        assert np.all(rec[1 + l, 1:] == 0.0)
    z = np.clip(rec[1:, 0], -P0.clamp_z, P0.clamp_z)
    SY = np.array([Sp[m] + O.driver(P0, i * dt, X[m], y1[m], z) * dt - cvi[m] for m in range(P0.M)])
    assert rec[0, 0] == pytest.approx(np.mean(SY), rel=1e-12, abs=1e-14)
    assert np.all(rec[0, 1:] == 0.0)
    assert math.isfinite(rec[0, 0])


def _network(n_in, n_out, H=64, seed=3):
    """Random network in the oracle's layout W1[H][in], b1, W2[H][H], b2, W3[out][H], b3."""
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(-1, 1, (H, n_in)) * math.sqrt(6.0 / (n_in + H)), rng.uniform(-0.2, 0.2, H),
             rng.uniform(-1, 1, (H, H)) * math.sqrt(6.0 / (2 * H)), rng.uniform(-0.2, 0.2, H),
             rng.uniform(-1, 1, (n_out, H)) * math.sqrt(6.0 / (H + n_out)), rng.uniform(-0.2, 0.2, n_out)]
    return np.concatenate([p.ravel() for p in parts])


NET_CASES = [
    ("logistic d=2 network stride 1", dict(d=2, N=5, lo=[-3.0] * 2, hi=[3.0] * 2, cells=[4, 4], M=64,
                                           driver=O.DRV_LOGISTIC, terminal=O.G_LOGISTIC), 1, 0),
    ("logistic d=3 network stride 2 centred", dict(d=3, N=5, lo=[-2.0] * 3, hi=[2.0] * 3, cells=[3, 2, 2], M=48,
                                                   driver=O.DRV_LOGISTIC, terminal=O.G_LOGISTIC), 2, 1),
]


@pytest.mark.parametrize("name,kw,stride,center", NET_CASES, ids=[c[0] for c in NET_CASES])
def test_flip_bound_covers_bfloat16_roundings_of_the_network(name, kw, stride, center):
    """With the control-variate network rounding its hidden activations to
    bfloat16, an activation within a few binary32 units of a rounding midpoint
    may round the other way in another precision.  The forced run rounds every
    such activation the other way (and takes every near-face look-up across
    its face): each coefficient must move by no more than the bound."""
    net = _network(kw["d"] + 1, kw["d"])
    bf = O.BF_WEIGHTS | O.BF_PAIR | O.BF_HIDDEN
    extra = dict(cv_params=net, cv_hidden=64, cv_bf16=bf, cv_stride=stride, z_center=center)
    P0 = _problem(kw, **extra)
    table, _ = O.solve(P0)
    K, i, eps = P0.K, 1, 1e-6
    bound = np.zeros(P0.table_shape())
    base = table.copy()
    O.solve(_problem(kw, face_eps=eps, flip_bound=bound, **extra), table=base, i_hi=i, i_lo=i)
    flipped = table.copy()
    O.solve(_problem(kw, face_eps=eps, face_flip=1, **extra), table=flipped, i_hi=i, i_lo=i)
    change = np.abs(flipped[i] - base[i])
    b = bound[i]
    scale = np.max(np.abs(base[i]))
    assert np.all(change <= b * (1 + 1e-6) + 1e-12 * scale), np.max(change - b)
    moved = change.reshape(K, -1).max(axis=1) > 1e-12 * scale
    assert moved.sum() >= K // 2, "most strata must meet an ambiguous rounding"
    ratio = change.reshape(K, -1).max(axis=1)[moved] / b.reshape(K, -1).max(axis=1)[moved]
    assert ratio.max() > 0.2, ratio
