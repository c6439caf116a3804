"""The learned control variate on the GPU: its network kernels against the
oracle's bfloat16 emulation of the same arithmetic, the training pairs and the
Adam step, the control-variate sweep against the oracle with the same frozen
network, and what the trained network gains (GPU tests; the library is called
through its C ABI).

Network arithmetic on both sides: bf16 weights, inputs as bf16 pairs
(hi + lo), bf16 hidden activations and gradient operands, binary32 (GPU) or
binary64 (oracle) sums, binary32 biases.  What remains between the two is the
summation order and the hardware exp2 / reciprocal of the GPU's SiLU, plus the
rare hidden activation whose bf16 rounding flips between a binary32 and a
binary64 pre-activation (one bf16 ulp, 2^-8 relative, on one unit); hence
norm-wise tolerances of 1e-3 for the network and elementwise 5e-3 of the
largest value.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from sides import oracle_problem, product_args

pytestmark = pytest.mark.gpu

H = 64
NET_BF = O.BF_WEIGHTS | O.BF_PAIR | O.BF_HIDDEN


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    return torch


def _params(n_in, n_out, seed, bias_scale=0.2):
    """Glorot weights from the library's initialiser plus random biases."""
    import paper_2407_21085_amd as S
    torch = _torch()
    p = S.mlp_init(n_in, n_out, seed)
    torch.cuda.synchronize()
    host = p.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(seed)
    o_b1 = H * n_in
    o_b2 = o_b1 + H + H * H
    o_b3 = o_b2 + H + n_out * H
    host[o_b1:o_b1 + H] = rng.normal(0, bias_scale, H)
    host[o_b2:o_b2 + H] = rng.normal(0, bias_scale, H)
    host[o_b3:o_b3 + n_out] = rng.normal(0, bias_scale, n_out)
    host = host.astype(np.float32).astype(np.float64)
    return torch.from_numpy(host.astype(np.float32)).cuda(), host


def _norm_rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


SHAPES = [(9, 8), (5, 4), (2, 1), (16, 16), (3, 13)]


@pytest.mark.parametrize("n_in,n_out", SHAPES, ids=[f"{a}to{b}" for a, b in SHAPES])
def test_mlp_forward_matches_oracle(n_in, n_out):
    import paper_2407_21085_amd as S
    torch = _torch()
    p_dev, p = _params(n_in, n_out, seed=n_in * 31 + n_out)
    rng = np.random.default_rng(5)
    n = 1000  # not a multiple of 64: a ragged last wavefront
    x = rng.normal(0, 1.5, (n, n_in)).astype(np.float32)
    _say(f"[gpu] mlp forward {n_in}->{n_out}")
    packed = S.mlp_pack(n_in, n_out, p_dev)
    y = S.mlp_forward(n_in, n_out, packed, torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    y = y.cpu().numpy().astype(np.float64)
    ref = O.mlp_forward(n_in, H, n_out, p, x.astype(np.float64), bf=NET_BF)
    err = _norm_rel(y, ref)
    _say(f"[gpu] forward norm-wise error {err:.2e}, max {np.max(np.abs(y - ref)):.2e}")
    assert err <= 1e-3
    assert np.max(np.abs(y - ref)) <= 5e-3 * np.max(np.abs(ref))
    # the emulation matters: the exact network differs by more than the tolerance
    exact = O.mlp_forward(n_in, H, n_out, p, x.astype(np.float64))
    assert _norm_rel(exact, ref) > err


def _groups(n_in, n_out):
    o = [0, H * n_in]
    o.append(o[-1] + H)
    o.append(o[-1] + H * H)
    o.append(o[-1] + H)
    o.append(o[-1] + n_out * H)
    o.append(o[-1] + n_out)
    names = ["W1", "b1", "W2", "b2", "W3", "b3"]
    return [(names[a], o[a], o[a + 1]) for a in range(6)]


@pytest.mark.parametrize("n_in,n_out", SHAPES, ids=[f"{a}to{b}" for a, b in SHAPES])
def test_mlp_backward_matches_oracle(n_in, n_out):
    import paper_2407_21085_amd as S
    torch = _torch()
    p_dev, p = _params(n_in, n_out, seed=7 * n_in + n_out)
    rng = np.random.default_rng(9)
    n = 2500  # three workgroups, the last one partial
    x = rng.normal(0, 1.5, (n, n_in)).astype(np.float32)
    dy = rng.normal(0, 1.0, (n, n_out)).astype(np.float32)
    _say(f"[gpu] mlp backward {n_in}->{n_out}")
    packed = S.mlp_pack(n_in, n_out, p_dev)
    g = S.mlp_backward(n_in, n_out, packed, torch.from_numpy(x).cuda(), torch.from_numpy(dy).cuda())
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    ref = O.mlp_backward(n_in, H, n_out, p, x.astype(np.float64), dy.astype(np.float64),
                         bf=O.BF_ALL)
    for name, a, b in _groups(n_in, n_out):
        err = _norm_rel(g[a:b], ref[a:b])
        _say(f"[gpu]   {name}: norm-wise error {err:.2e}")
        assert err <= 2e-3, name


def test_mlp_backward_zero_samples_gives_zero_gradient():
    import paper_2407_21085_amd as S
    torch = _torch()
    p_dev, _ = _params(5, 4, seed=1)
    packed = S.mlp_pack(5, 4, p_dev)
    g = S.mlp_backward(5, 4, packed, torch.zeros((0, 5), device="cuda"), torch.zeros((0, 4), device="cuda"))
    torch.cuda.synchronize()
    assert float(g.abs().max()) == 0.0


def _pairs(n, n_in, n_out, seed, target):
    rng = np.random.default_rng(seed)
    x16 = np.zeros((n, 16), dtype=np.float32)
    z16 = np.zeros((n, 16), dtype=np.float32)
    x16[:, :n_in] = rng.normal(0, 1.0, (n, n_in))
    z16[:, :n_out] = target(x16[:, :n_in])
    return x16, z16


@pytest.mark.parametrize("batch", [256, 1024])
def test_mlp_train_step_gradient_and_adam(batch):
    """One Adam step from zero moments: m = (1 - beta1) g, v = (1 - beta2) g^2 with
    g the gradient of the batch loss mean_s sum_o (z_theta - z)^2, which the
    oracle computes from its forward pass (dy = 2 (y - z) / batch) and its
    backward pass.  The parameter step is then lr m_hat / (sqrt(v_hat) + eps).
    A batch of 1024 spreads the gradient over four workgroups."""
    import paper_2407_21085_amd as S
    torch = _torch()
    n_in, n_out = 5, 4
    p_dev, p = _params(n_in, n_out, seed=3)
    x16, z16 = _pairs(2048, n_in, n_out, 4, lambda x: 0.3 * np.tanh(x[:, :n_out]))
    cfg = S.TrainConfig(updates_per_step=1, batch=batch, lr=1e-3)
    m = torch.zeros_like(p_dev)
    v = torch.zeros_like(p_dev)
    p0 = p_dev.clone()
    _say(f"[gpu] mlp train: one Adam step, batch {batch}")
    packed, loss = S.mlp_train(n_in, n_out, p_dev, m, v, 0, torch.from_numpy(x16).cuda(),
                               torch.from_numpy(z16).cuda(), cfg)
    torch.cuda.synchronize()
    g_gpu = m.cpu().numpy().astype(np.float64) / (1 - cfg.beta1)
    xb = x16[:batch, :n_in].astype(np.float64)
    zb = z16[:batch, :n_out].astype(np.float64)
    y = O.mlp_forward(n_in, H, n_out, p, xb, bf=NET_BF)
    dy = 2.0 * (y - zb) / batch
    g_ref = O.mlp_backward(n_in, H, n_out, p, xb, dy, bf=O.BF_ALL)
    for name, a, b in _groups(n_in, n_out):
        err = _norm_rel(g_gpu[a:b], g_ref[a:b])
        _say(f"[gpu]   {name}: gradient norm-wise error {err:.2e}")
        assert err <= 2e-3, name
    loss_ref = float(np.mean(np.sum((y - zb) ** 2, axis=1)))
    assert float(loss.cpu()[0]) == pytest.approx(loss_ref, rel=1e-3)
    mm, vv = m.cpu().numpy(), v.cpu().numpy()
    np.testing.assert_allclose(vv, (1 - cfg.beta2) * (g_gpu.astype(np.float32)) ** 2, rtol=1e-4, atol=1e-20)
    step = cfg.lr * (mm / (1 - cfg.beta1)) / (np.sqrt(vv / (1 - cfg.beta2)) + cfg.eps)
    np.testing.assert_allclose(p0.cpu().numpy() - p_dev.cpu().numpy(), step, rtol=1e-3, atol=1e-9)
    # the returned packed network is the packing of the updated parameters
    np.testing.assert_array_equal(packed.cpu().numpy(), S.mlp_pack(n_in, n_out, p_dev).cpu().numpy())


def test_mlp_train_updates_chain_in_place():
    """Three updates in one call equal three calls of one update each (Adam step
    counts 0, 1, 2 and the pairs each update takes), bit for bit: each update
    reads the packed network the previous one rewrote, which must equal the
    packing of the updated parameters."""
    import paper_2407_21085_amd as S
    torch = _torch()
    n_in, n_out, batch = 9, 8, 512
    x16, z16 = _pairs(4096, n_in, n_out, 21, lambda x: 0.2 * np.sin(x[:, :n_out]))
    xd, zd = torch.from_numpy(x16).cuda(), torch.from_numpy(z16).cuda()
    p_a, _ = _params(n_in, n_out, seed=22)
    p_b = p_a.clone()
    m_a, v_a = torch.zeros_like(p_a), torch.zeros_like(p_a)
    m_b, v_b = torch.zeros_like(p_a), torch.zeros_like(p_a)
    _say("[gpu] mlp train: three updates in one call and in three")
    packed_a, loss_a = S.mlp_train(n_in, n_out, p_a, m_a, v_a, 0, xd, zd,
                                   S.TrainConfig(updates_per_step=3, batch=batch, lr=2e-3))
    losses = []
    for u in range(3):
        packed_b, lb = S.mlp_train(n_in, n_out, p_b, m_b, v_b, u, xd[u * batch:], zd[u * batch:],
                                   S.TrainConfig(updates_per_step=1, batch=batch, lr=2e-3))
        losses.append(lb)
    torch.cuda.synchronize()
    assert torch.equal(p_a, p_b) and torch.equal(m_a, m_b) and torch.equal(v_a, v_b)
    assert torch.equal(packed_a, packed_b)
    assert torch.equal(loss_a, torch.cat(losses))


def test_mlp_training_fits_a_smooth_target():
    import paper_2407_21085_amd as S
    torch = _torch()
    n_in, n_out = 5, 4
    p_dev = S.mlp_init(n_in, n_out, 11, zero_output_layer=True)
    target = lambda x: 0.25 / np.cosh(x[:, :1] + x[:, 1:2]) ** 2 + 0.1 * x[:, :n_out]  # noqa: E731
    x16, z16 = _pairs(8192, n_in, n_out, 12, target)
    m = torch.zeros_like(p_dev)
    v = torch.zeros_like(p_dev)
    cfg = S.TrainConfig(updates_per_step=400, batch=512, lr=3e-3)
    _say("[gpu] mlp train: 400 Adam steps")
    _, loss = S.mlp_train(n_in, n_out, p_dev, m, v, 0, torch.from_numpy(x16).cuda(),
                          torch.from_numpy(z16).cuda(), cfg)
    torch.cuda.synchronize()
    loss = loss.cpu().numpy()
    _say(f"[gpu] loss {loss[0]:.3e} -> {loss[-20:].mean():.3e}")
    assert np.all(np.isfinite(loss))
    assert loss[-20:].mean() < 0.05 * loss[0]


# ------------------------------------------------------- training pairs

def test_cv_pairs_match_oracle_draws():
    """Pair s: stratum floor(K u0), simulation floor(M u1) from the Philox words of
    counter (0, s, 0xFFFFFFFE, tag); the start point of that simulation (the
    sweep's own draw) and the fitted z_i of the stratum there."""
    import paper_2407_21085_amd as S
    torch = _torch()
    cfg = dict(W.config("cfg2"), N=6, cells=[4] * 4, M=32, instance=3)
    K = 4 ** 4
    P, G, Opt = product_args(cfg)
    rng = np.random.default_rng(2)
    table = rng.normal(0, 0.3, (cfg["N"], K, 5, 5)).astype(np.float32)
    i, n = 2, 300
    _say("[gpu] training pairs")
    x16, z16 = S.cv_pairs(P, G, Opt, torch.from_numpy(table).cuda(), i, n)
    torch.cuda.synchronize()
    x16, z16 = x16.cpu().numpy(), z16.cpu().numpy()
    Po = oracle_problem(cfg)
    seed = cfg["seed"]
    tag = (i & 0xFFFF) | (cfg["instance"] << 16)
    key = (seed & 0xFFFFFFFF, seed >> 32)
    dt = cfg["T"] / cfg["N"]
    t64 = table.astype(np.float64)
    for s in range(n):
        w = O.philox4x32_10((0, s, 0xFFFFFFFE, tag), key)
        k = (int(w[0]) * K) >> 32
        m = (int(w[1]) * cfg["M"]) >> 32
        x = O.start_point(Po, i, k, m)
        _, z = O.evaluate(Po, t64, i, x)
        assert x16[s, 0] == pytest.approx(i * dt, rel=1e-7)
        np.testing.assert_allclose(x16[s, 1:5], x, rtol=2e-5, atol=2e-5)
        np.testing.assert_array_equal(x16[s, 5:], 0.0)
        np.testing.assert_allclose(z16[s, :4], z[0], rtol=1e-4, atol=1e-5)
        np.testing.assert_array_equal(z16[s, 4:], 0.0)


# ------------------------------------------------- sweeps with the network

def _cv_oracle(cfg, params, i_hi, i_lo, eps, stride, center):
    """Oracle steps with the frozen network, the near-face flags and the flip
    bound (face flips and ambiguous bfloat16 roundings of the network)."""
    K = int(np.prod(cfg["cells"]))
    f_orc = np.zeros((cfg["N"], K), dtype=np.uint8)
    P = oracle_problem(cfg, face_flags=f_orc, face_eps=eps)
    P.cv_params = params
    P.cv_hidden = H
    P.cv_bf16 = NET_BF
    P.cv_stride = stride
    P.z_center = int(center)
    P.flip_bound = np.zeros(P.table_shape())
    orc, _ = O.solve(P, i_hi=i_hi, i_lo=i_lo)
    return orc, f_orc, P.flip_bound


def cv_step_parity(cfg, steps, params_dev, params, eps=2e-6, stride=1, center=False, tol=2e-4):
    """Backward step i of the library with the frozen network against the
    oracle's step i with the same network, both from the oracle's rows > i.
    Returns (worst excess of |gpu - orc| over tol ref + flip bound, which
    must be <= 0; worst error relative to ref on strata without a near-face
    look-up; flagged share; RMS relative error)."""
    import paper_2407_21085_amd as S
    from test_gpu_parity import bounded_parity
    torch = _torch()
    K = int(np.prod(cfg["cells"]))
    orc, f_orc, bound = _cv_oracle(cfg, params, cfg["N"] - 1, min(steps), eps, stride, center)
    worst, excess, shares, rms = 0.0, -np.inf, [], 0.0
    for i in steps:
        table = torch.from_numpy(orc).to(torch.float32).cuda()
        f_gpu = torch.zeros((cfg["N"], K), dtype=torch.uint8, device="cuda")
        Pp, G, Opt = product_args(cfg, step_hi=i, step_lo=i)
        Opt.face_flags, Opt.face_eps = f_gpu, eps
        Opt.cv, Opt.cv_params, Opt.cv_stride = S.CV_FROZEN, params_dev, stride
        if center:
            Opt.flags |= S.F_CV_CENTER_Z
        _say(f"[gpu] {cfg['name']} with the frozen network (stride {stride}, centre {center}): step {i}")
        S.solve(Pp, G, Opt, table=table)
        torch.cuda.synchronize()
        flags = f_orc | f_gpu.cpu().numpy()
        gpu = table.double().cpu().numpy()
        e, x = bounded_parity(gpu, orc, bound, [i], flags, tol)
        worst, excess = max(worst, e), max(excess, x)
        shares.append(float(flags[i].mean()))
        keep = flags[i] == 0
        for c in range(orc.shape[2]):
            ref = np.sqrt(np.mean(orc[i, keep, c, :] ** 2))
            rms = max(rms, float(np.sqrt(np.mean((gpu[i, keep, c, :] - orc[i, keep, c, :]) ** 2)) / ref))
    _say(f"[gpu] frozen-network per-step parity: max {worst:.3e}, RMS {rms:.3e}, flagged share "
         f"{max(shares):.4f}, worst excess over tol + flip bound {excess:.3e}")
    return excess, worst, max(shares), rms


CV_CASES = [
    # d = 4 logistic problem, K = 4^4, M = 32 (two strata per wavefront, four wavefronts per workgroup)
    ("d4 lp1", dict(N=6, cells=[4] * 4, M=32, lanes=0)),
    # 8 lanes per stratum (eight strata per wavefront), K = 3^4 = 81 (ragged last workgroup)
    ("d4 lp1 8 lanes", dict(N=5, cells=[3] * 4, M=24, lanes=8)),
    ("d4 lp0", dict(N=5, cells=[4] * 4, M=16, basis="LP0")),
    # M not a multiple of the lanes: the lanes past simulation M-1 make a last trip and discard it
    ("d4 lp1 M=20 32 lanes", dict(N=5, cells=[3] * 4, M=20)),
    ("d4 lp1 M=40 16 lanes", dict(N=5, cells=[4] * 4, M=40, lanes=16)),
    # strata over two and four wavefronts
    ("d4 lp1 M=100 128 lanes", dict(N=4, cells=[3] * 4, M=100)),
    ("d8 lp1 M=160 256 lanes stride 2 centred", dict(d=8, N=3, lo=[-3.0] * 8, hi=[3.0] * 8, cells=[2] * 8,
                                                     M=160, cv_stride=2, center=True)),
    ("d8 lp1", dict(d=8, N=4, lo=[-3.0] * 8, hi=[3.0] * 8, cells=[2] * 8, M=64)),
    ("d2 cos linear kappa", dict(d=2, N=6, lo=[-2.0] * 2, hi=[2.0] * 2, cells=[6, 5], M=40,
                                 driver="linear", terminal="cos", r=0.2, kappa=0.3)),
    ("d3 clamps", dict(d=3, N=5, lo=[-2.0] * 3, hi=[2.0] * 3, cells=[3, 4, 2], M=48,
                       clamp_y=0.7, clamp_z=0.2)),
    ("d4 lp1 stride 3 centred", dict(N=8, cells=[4] * 4, M=32, cv_stride=3, center=True)),
    ("d8 lp1 stride 2 centred", dict(d=8, N=5, lo=[-3.0] * 8, hi=[3.0] * 8, cells=[2] * 8, M=64,
                                     cv_stride=2, center=True)),
    ("d3 clamps centred", dict(d=3, N=5, lo=[-2.0] * 3, hi=[2.0] * 3, cells=[3, 4, 2], M=48,
                               clamp_y=0.7, clamp_z=0.2, center=True)),
    # equal-probability cells (unbounded outer cells), truncated y, centred, stride 2
    ("d4 lp1 equal probability centred", dict(N=6, lo=None, hi=None, grid_kind=1, cells=[3, 4, 3, 2], M=32,
                                              clamp_y=1.0, cv_stride=2, center=True)),
]


@pytest.mark.parametrize("name,kw", CV_CASES, ids=[c[0] for c in CV_CASES])
def test_frozen_network_sweep_step_parity(name, kw):
    """Per-step parity of the control-variate sweep with a frozen random network.

    The network rounds its hidden activations to bf16, and a binary32
    activation (GPU) and a binary64 one (oracle) that straddle a rounding
    midpoint round to neighbouring bf16 values: about one network evaluation
    in fifty.  One such flip moves z_theta by about |W3| 2^-8 |h| ~ 3e-4, and
    the z response multiplies the control-variate sum by dW_i / dt.  The
    oracle bounds, per coefficient, what rounding every ambiguous activation
    (within 32 binary32 units of a midpoint) the other way can change, as it
    does for near-face look-ups; every coefficient must lie within 2e-4 of
    the largest (the plain binary32 bound) plus that bound, and the RMS
    relative error within 2e-4 (observed at most 1.2e-4).  A wrong index,
    time, stride or centre (errors of order one) would exceed both by far."""
    kw = dict(kw)
    stride, center = kw.pop("cv_stride", 1), kw.pop("center", False)
    cfg = dict(W.config("cfg2"), name=name, seed=17, **kw)
    d = cfg["d"]
    params_dev, params = _params(d + 1, d, seed=23 + d)
    steps = sorted({cfg["N"] - 1, cfg["N"] - 2, 1, 0}, reverse=True)
    # equal-probability cells: the binary32 coordinate C F(x) carries a few ulps of exp and division
    eps = 2e-5 if cfg.get("grid_kind") else 2e-6
    excess, err, share, rms = cv_step_parity(cfg, steps, params_dev, params, eps=eps, stride=stride,
                                             center=center)
    assert rms <= 2e-4
    assert excess <= 0.0
    assert share < 0.1


def test_frozen_network_with_zero_output_equals_plain_sweep():
    """A network whose output layer is zero subtracts nothing: the sweep with it
    is bit-identical to the plain sweep (same draws, same arithmetic outside the
    network)."""
    import paper_2407_21085_amd as S
    torch = _torch()
    cfg = dict(W.config("cfg2"), N=5, cells=[4] * 4, M=32)
    P, G, Opt = product_args(cfg)
    plain, _ = S.solve(P, G, Opt)
    params = S.mlp_init(5, 4, 3, zero_output_layer=True)
    Opt.cv, Opt.cv_params = S.CV_FROZEN, params
    with_net, _ = S.solve(P, G, Opt)
    torch.cuda.synchronize()
    assert torch.equal(plain, with_net)


def test_frozen_zero_network_at_headline_size_matches_plain_sweep():
    """At the headline size (K = 4^8, M = 64, N = 50, binary32) the sweep with a
    zero-output network subtracts nothing and gives the plain sweep's rows bit
    for bit where the plain sweep runs the plain path loop or the loop with one
    gather in flight (steps 49..14, paths of up to 36 steps; the control-variate
    kernel keeps the plain loop).  From 176 MiB of look-up rows (steps 13..0)
    the plain sweep keeps two gathers in flight, the same arithmetic compiled
    otherwise: there every record agrees to 1e-4 of its largest coefficient."""
    import paper_2407_21085_amd as S
    torch = _torch()
    cfg = W.config("cfg5")
    P, G, Opt = product_args(cfg)
    _say("[gpu] headline size: plain sweep and the sweep with a zero-output network")
    plain, _ = S.solve(P, G, Opt)
    Opt.cv, Opt.cv_params = S.CV_FROZEN, S.mlp_init(cfg["d"] + 1, cfg["d"], 5, zero_output_layer=True)
    with_net, _ = S.solve(P, G, Opt)
    torch.cuda.synchronize()
    assert torch.equal(plain[14:], with_net[14:])
    a, b = plain[:14].double(), with_net[:14].double()
    scale = a.abs().amax(dim=(2, 3), keepdim=True)
    assert float(((a - b).abs() / scale).max()) <= 1e-4


def _logistic_exact(t, x):
    s = np.sum(x, axis=-1) + t
    u = 1.0 / (1.0 + np.exp(-s))
    return u, u * (1.0 - u)


def _grid_errors(S, P, G, Opt, table, cfg, i, n=4096, seed=0):
    """RMS errors of the fitted y_i, z_i against the closed form at points drawn
    from the sampling law restricted to the central quarter of the domain."""
    torch = _torch()
    rng = np.random.default_rng(seed)
    d = cfg["d"]
    x = rng.uniform(-1.5, 1.5, (n, d))
    y, z = S.evaluate(P, G, Opt.basis, Opt.prec, table, i, torch.from_numpy(x).cuda())
    torch.cuda.synchronize()
    t = i * cfg["T"] / cfg["N"]
    u, zu = _logistic_exact(t, x)
    ey = float(np.sqrt(np.mean((y.cpu().numpy() - u) ** 2)))
    ez = float(np.sqrt(np.mean((z.cpu().numpy() - zu[:, None]) ** 2)))
    return ey, ez


def test_online_network_reduces_the_error_of_the_fits():
    """The d = 4 logistic problem with N = 50 steps and M = 32 simulations per
    stratum: the online control variate (network trained on the sweep's own
    pairs) against the plain estimator, same draws.  The network's terms have
    conditional mean zero, so both estimate the same coefficients; the test
    checks that the one with the trained network is closer to the closed form
    (y and z at t = 0 and mid-way), over three seeds, and that training
    reduced its loss."""
    import paper_2407_21085_amd as S
    torch = _torch()
    cfg = W.config("cfg4")
    res = {"plain": [], "cv": []}
    for seed in (1, 2, 3):
        P, G, Opt = product_args(cfg, seed=seed)
        _say(f"[gpu] cfg4 plain seed {seed}")
        tab_plain, _ = S.solve(P, G, Opt)
        params = S.mlp_init(5, 4, 100 + seed, zero_output_layer=True)
        Opt.cv, Opt.cv_params = S.CV_ONLINE, params
        Opt.flags |= S.F_CV_CENTER_Z
        Opt.cv_train = S.TrainConfig(updates_per_step=16, batch=512, lr=2e-3)
        _say(f"[gpu] cfg4 online control variate seed {seed}")
        tab_cv, st = S.solve(P, G, Opt)
        torch.cuda.synchronize()
        _say(f"[gpu]   training loss {st['cv_loss_first']:.3e} -> {st['cv_loss_last']:.3e}")
        assert math.isfinite(st["cv_loss_last"]) and math.isfinite(st["cv_loss_first"])
        for name, tab in (("plain", tab_plain), ("cv", tab_cv)):
            errs = [_grid_errors(S, P, G, Opt, tab, cfg, i, seed=seed) for i in (0, 25)]
            res[name].append(errs)
            _say(f"[gpu]   {name}: (y, z) RMS errors at t=0, 0.5: {errs}")
    plain = np.array(res["plain"])
    cv = np.array(res["cv"])
    ratio = np.mean(plain ** 2, axis=0) / np.mean(cv ** 2, axis=0)
    _say(f"[gpu] MSE ratio plain / control variate, [(y, z) at t=0, t=0.5]: {ratio.tolist()}")
    assert np.all(ratio[:, 0] > 1.5)
    assert np.all(ratio[:, 1] > 1.5)


def test_frozen_network_sweep_graph_replays():
    """The control-variate sweep (frozen network, stride 2, centred) captured in a
    hipGraph: three replays, each equal to the eager sweep."""
    import paper_2407_21085_amd as S
    torch = _torch()
    cfg = dict(W.config("cfg2"), N=6, cells=[4] * 4, M=32)
    P, G, Opt = product_args(cfg)
    params = S.mlp_init(5, 4, 7)
    Opt.cv, Opt.cv_params, Opt.cv_stride = S.CV_FROZEN, params, 2
    Opt.flags |= S.F_CV_CENTER_Z
    eager, _ = S.solve(P, G, Opt)
    Opt.flags |= S.F_GRAPH
    stream = torch.cuda.Stream()
    ws = S.srmdp.alloc_workspace(P, G, Opt)
    table = torch.zeros_like(eager)
    for rep in range(3):
        table.zero_()
        torch.cuda.synchronize()
        _say(f"[gpu] control-variate graph replay {rep}")
        with torch.cuda.stream(stream):
            S.solve(P, G, Opt, table=table, workspace=ws, stream=stream, stats=False)
        torch.cuda.synchronize()
        assert torch.equal(table, eager)
    S.release_graphs()


@pytest.mark.parametrize("mode", ["plain", "online"])
def test_sweep_reads_nothing_it_did_not_write(mode):
    """A sweep's result does not depend on what its table and workspace held
    before: a workspace and table filled with 0xFF bytes (NaN patterns) and
    zero-filled ones give the same table, bit for bit, with the online control
    variate (network, Adam state, training pairs and gradient partials all in
    the workspace) and without it."""
    import paper_2407_21085_amd as S
    torch = _torch()
    cfg = dict(W.config("cfg2"), N=6, cells=[4] * 4, M=40)
    tables = []
    for fill in (0x00, 0xFF):
        P, G, Opt = product_args(cfg)
        if mode == "online":
            Opt.cv, Opt.cv_stride = S.CV_ONLINE, 2
            Opt.flags |= S.F_CV_CENTER_Z
            Opt.cv_train = S.TrainConfig(updates_per_step=2, batch=512, lr=1e-2)
            Opt.cv_params = S.mlp_init(5, 4, 9, zero_output_layer=True)
        ws = S.srmdp.alloc_workspace(P, G, Opt)
        table = S.srmdp.alloc_table(P, G, Opt)
        ws.fill_(fill)
        table.view(torch.uint8).fill_(fill)
        torch.cuda.synchronize()
        _say(f"[gpu] {mode} sweep on a workspace filled with {fill:#04x}")
        S.solve(P, G, Opt, table=table, workspace=ws)
        torch.cuda.synchronize()
        tables.append(table)
    assert bool(torch.isfinite(tables[1]).all())
    assert torch.equal(tables[0], tables[1])


def test_control_variate_keeps_the_mean_of_the_fits():
    """Unbiasedness: with a linear driver (f = -r y + kappa sum z) the fitted
    coefficients are linear in the responses, so their expectation is the same
    with and without the network's martingale terms and the centring.  Over 16
    seeds, the mean difference (control variate - plain) of the coefficients,
    averaged per step and component over strata and basis functions, stays
    within 4 standard errors of zero, while single runs do change (the
    control variate changes the noise)."""
    import paper_2407_21085_amd as S
    torch = _torch()
    cfg = dict(W.config("cfg1"), d=2, N=6, lo=[-2.0] * 2, hi=[2.0] * 2, cells=[6, 6], M=32, prec="fp32",
               driver="linear", terminal="cos", r=0.2, kappa=0.3)
    params = S.mlp_init(3, 2, 11)
    diffs = []
    for seed in range(1, 17):
        P, G, Opt = product_args(cfg, seed=seed)
        plain, _ = S.solve(P, G, Opt)
        Opt.cv, Opt.cv_params, Opt.cv_stride = S.CV_FROZEN, params, 2
        Opt.flags |= S.F_CV_CENTER_Z
        cv, _ = S.solve(P, G, Opt)
        torch.cuda.synchronize()
        d = (cv - plain).double().cpu().numpy()
        diffs.append(d.mean(axis=(1, 3)))  # per (step, component)
    diffs = np.array(diffs)
    mean = diffs.mean(axis=0)
    se = diffs.std(axis=0, ddof=1) / math.sqrt(diffs.shape[0])
    _say(f"[gpu] mean difference / standard error per (step, component): {np.round(mean / se, 2).tolist()}")
    assert np.all(np.abs(mean) <= 4.0 * se)
    assert np.all(diffs.std(axis=0) > 0)  # the network does change every run
