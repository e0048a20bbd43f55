"""Pins of the oracle's FP64 surrogate network: the analytic gradient of the
batch MSE against central finite differences of the forward pass, and the
forward pass against a direct numpy evaluation of the layer formulas."""
import numpy as np

import oracle


def _params(seed):
    rng = np.random.default_rng(seed)
    p = rng.uniform(-1, 1, oracle.MLP_NPARAM) * 0.3
    return p


def _numpy_forward(p, x):
    o = 0
    W1 = p[o:o + 192].reshape(64, 3); o += 192
    b1 = p[o:o + 64]; o += 64
    W2 = p[o:o + 4096].reshape(64, 64); o += 4096
    b2 = p[o:o + 64]; o += 64
    W3 = p[o:o + 4096].reshape(64, 64); o += 4096
    b3 = p[o:o + 64]; o += 64
    W4 = p[o:o + 256].reshape(4, 64); o += 256
    b4 = p[o:o + 4]
    silu = lambda z: z / (1 + np.exp(-z))
    h = silu(x @ W1.T + b1)
    h = silu(h @ W2.T + b2)
    h = silu(h @ W3.T + b3)
    return h @ W4.T + b4


def test_forward_matches_layer_formulas():
    p = _params(0)
    x = np.random.default_rng(1).uniform(-1, 1, (50, 3))
    np.testing.assert_allclose(oracle.mlp_forward(p, x), _numpy_forward(p, x), rtol=1e-12, atol=1e-13)


def test_gradient_vs_central_differences():
    p = _params(2)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (16, 3))
    t = rng.normal(size=(16, 4))
    loss, g = oracle.mlp_grad(p, x, t)
    y = oracle.mlp_forward(p, x)
    assert abs(loss - ((y - t) ** 2).mean()) < 1e-14 * max(1.0, loss)
    idx = np.concatenate([rng.choice(8836, 200, replace=False), [0, 191, 192, 255, 8831, 8835]])
    eps = 1e-6
    for i in idx:
        q = p.copy()
        q[i] += eps
        lp = ((oracle.mlp_forward(q, x) - t) ** 2).mean()
        q[i] -= 2 * eps
        lm = ((oracle.mlp_forward(q, x) - t) ** 2).mean()
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g).max()), i
