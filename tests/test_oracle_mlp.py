"""Pin of the oracle's network (the learned control variate's z_theta):
parameter gradients against central finite differences of the forward pass,
and the forward pass against a layer-by-layer numpy evaluation."""
import numpy as np
import pytest

import oracle as O


def _setup(n_in=5, H=16, n_out=4, B=7, seed=0):
    rng = np.random.default_rng(seed)
    n = O.mlp_param_count(n_in, H, n_out)
    assert n == H * n_in + H + H * H + H + n_out * H + n_out
    p = rng.normal(0, 0.4, n)
    x = rng.normal(0, 1, (B, n_in))
    dy = rng.normal(0, 1, (B, n_out))
    return n_in, H, n_out, p, x, dy


def test_forward_matches_numpy_layers():
    n_in, H, n_out, p, x, _ = _setup()
    W1 = p[:H * n_in].reshape(H, n_in); o = H * n_in
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + n_out * H].reshape(n_out, H); o += n_out * H
    b3 = p[o:o + n_out]
    silu = lambda a: a / (1 + np.exp(-a))
    ref = silu(silu(x @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    np.testing.assert_allclose(O.mlp_forward(n_in, H, n_out, p, x), ref, rtol=1e-13, atol=1e-14)


def test_gradient_matches_central_differences():
    n_in, H, n_out, p, x, dy = _setup()
    g = O.mlp_backward(n_in, H, n_out, p, x, dy)
    eps = 1e-6
    fd = np.empty_like(p)
    for a in range(p.size):
        pp, pm = p.copy(), p.copy()
        pp[a] += eps
        pm[a] -= eps
        fd[a] = (np.sum(dy * O.mlp_forward(n_in, H, n_out, pp, x)) -
                 np.sum(dy * O.mlp_forward(n_in, H, n_out, pm, x))) / (2 * eps)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-8)


def test_bf16_rounding_is_round_to_nearest_even():
    # 1 + 2^-8 is exactly halfway between bf16 neighbours 1 and 1 + 2^-7: ties to even (1)
    n_in, H, n_out = 1, 1, 1
    # a network that returns its input: W1 = 1, b1 = 0 ... not available (SiLU), so check the
    # input rounding through a zero-weight first layer and a bias-only output
    p = np.zeros(O.mlp_param_count(n_in, H, n_out))
    x = np.array([[1.0 + 2.0 ** -8], [1.0 + 3 * 2.0 ** -8]])
    # forward with weights 1 in layer 1 picks up the rounded input: y = b3 + W3 silu(W2 silu(W1 x))
    p[0] = 1.0                      # W1
    p[2] = 1.0                      # W2
    p[4] = 1.0                      # W3
    y_exact = O.mlp_forward(n_in, H, n_out, p, x)
    y_round = O.mlp_forward(n_in, H, n_out, p, x, bf=O.BF_INPUT)
    x_r = np.array([[1.0], [1.0 + 4 * 2.0 ** -8]])  # ties to even
    np.testing.assert_allclose(y_round, O.mlp_forward(n_in, H, n_out, p, x_r), rtol=1e-15)
    assert not np.allclose(y_exact, y_round)


def test_bf16_emulated_gradient_matches_central_differences_of_its_forward():
    """With weights and inputs rounded (not the hidden values, whose rounding is
    piecewise constant), the emulated backward is the exact gradient of the
    emulated forward with respect to the biases and the output layer."""
    n_in, H, n_out, p, x, dy = _setup(seed=3)
    bf = O.BF_WEIGHTS | O.BF_INPUT
    g = O.mlp_backward(n_in, H, n_out, p, x, dy, bf=bf)
    n = p.size
    o_b3 = n - n_out
    eps = 1e-6
    for a in list(range(o_b3, n)) + [H * n_in + 3]:   # output biases and one first-layer bias
        pp, pm = p.copy(), p.copy()
        pp[a] += eps
        pm[a] -= eps
        fd = (np.sum(dy * O.mlp_forward(n_in, H, n_out, pp, x, bf=bf)) -
              np.sum(dy * O.mlp_forward(n_in, H, n_out, pm, x, bf=bf))) / (2 * eps)
        assert g[a] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_bf16_pair_input_keeps_sixteen_bits():
    """Input as hi + lo with hi = bf16(x), lo = bf16(x - hi): worked values.
    x = 1 + 2^-8 + 2^-12: hi = 1 + 2^-7 (above the tie), lo = bf16(2^-12 - 2^-8) = -(2^-8 - 2^-12)
    exactly (5 significant bits), so the pair is exact.  x = 3 + 2^-20 (binary32 exact): hi = 3,
    lo = 2^-20 exactly.  x = 1 + 2^-9 + 2^-17 + 2^-19: hi = 1, lo = bf16(2^-9 + 2^-17 + 2^-19);
    the ulp of lo is 2^-16 and the tail is 0.625 ulp, so lo = 2^-9 + 2^-16."""
    n_in, H, n_out = 1, 1, 1
    p = np.zeros(O.mlp_param_count(n_in, H, n_out))
    p[0] = 1.0
    p[2] = 1.0
    p[4] = 1.0
    xs = np.array([[1 + 2.0 ** -8 + 2.0 ** -12], [3 + 2.0 ** -20], [1 + 2.0 ** -9 + 2.0 ** -17 + 2.0 ** -19]])
    eff = np.array([[1 + 2.0 ** -8 + 2.0 ** -12], [3 + 2.0 ** -20], [1 + 2.0 ** -9 + 2.0 ** -16]])
    y_pair = O.mlp_forward(n_in, H, n_out, p, xs, bf=O.BF_PAIR)
    np.testing.assert_allclose(y_pair, O.mlp_forward(n_in, H, n_out, p, eff), rtol=1e-15)
    # a single bf16 would lose the low bits
    assert not np.allclose(O.mlp_forward(n_in, H, n_out, p, xs, bf=O.BF_INPUT), y_pair, rtol=1e-6)
