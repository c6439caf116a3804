"""Pin of the oracle's network (the learned control variate's z_theta):
parameter gradients against central finite differences of the forward pass,
and the forward pass against a layer-by-layer numpy evaluation."""
import numpy as np

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
