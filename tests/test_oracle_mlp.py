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
    W4 = p[o:o + 640].reshape(10, 64); o += 640
    b4 = p[o:o + 10]
    def act(z):
        t = np.clip(z / 6 + 0.5, 0, 1)
        return z * t * t * (3 - 2 * t)
    h = act(x @ W1.T + b1)
    h = act(h @ W2.T + b2)
    h = act(h @ W3.T + b3)
    return h @ W4.T + b4


def _chain_params():
    """A network whose output 0 is f(f(f(x0))) for the activation f: one path
    of unit weights through neuron 0 of every layer, everything else zero."""
    p = np.zeros(oracle.MLP_NPARAM)
    p[0] = 1.0                      # W1[0][0]
    p[256] = 1.0                    # W2[0][0]
    p[256 + 4096 + 64] = 1.0        # W3[0][0]
    p[256 + 2 * (4096 + 64)] = 1.0  # W4[0][0]
    return p


def test_forward_matches_layer_formulas():
    p = _params(0)
    x = np.random.default_rng(1).uniform(-1, 1, (50, 3))
    np.testing.assert_allclose(oracle.mlp_forward(p, x), _numpy_forward(p, x), rtol=1e-12, atol=1e-13)


def test_gradient_vs_central_differences():
    p = _params(2)
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (16, 3))
    t = rng.normal(size=(16, oracle.MLP_NOUT))
    loss, g = oracle.mlp_grad(p, x, t)
    y = oracle.mlp_forward(p, x)
    assert abs(loss - ((y - t) ** 2).mean()) < 1e-14 * max(1.0, loss)
    n = oracle.MLP_NPARAM
    idx = np.concatenate([rng.choice(n, 200, replace=False), [0, 191, 192, 255, n - 650, n - 11, n - 10, n - 1]])
    eps = 1e-6
    for i in idx:
        q = p.copy()
        q[i] += eps
        lp = ((oracle.mlp_forward(q, x) - t) ** 2).mean()
        q[i] -= 2 * eps
        lm = ((oracle.mlp_forward(q, x) - t) ** 2).mean()
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g).max()), i


def test_activation_special_values():
    """f(z) = z for z >= 3, 0 for z <= -3, f(1) = 20/27 (t = 2/3, S = 20/27),
    f(-1) = -7/27 (t = 1/3, S = 7/27), f(0) = 0; checked through a chain of
    three activations."""
    p = _chain_params()
    x = np.array([[5.0, 0, 0], [3.0, 0, 0], [-4.0, 0, 0], [0.0, 0, 0], [1.0, 0, 0]])
    y = oracle.mlp_forward(p, x)[:, 0]
    f1 = 20 / 27
    t = f1 / 6 + 0.5
    f2 = f1 * t * t * (3 - 2 * t)
    t = f2 / 6 + 0.5
    f3 = f2 * t * t * (3 - 2 * t)
    np.testing.assert_allclose(y, [5.0, 3.0, 0.0, 0.0, f3], rtol=0, atol=1e-15)
    # one layer only: W2 and W3 paths replaced by exact pass-through of z >= 3
    q = _chain_params()
    q[192] = 10.0                   # b1[0]: pre-activation 10 + x0 stays > 3
    y = oracle.mlp_forward(q, np.array([[-1.0, 0, 0]]))[0, 0]
    assert y == 9.0
    # f(-1) through the first layer, then shifted up by +10 in layer 2
    q = _chain_params()
    q[256 + 4096] = 10.0            # b2[0]
    y = oracle.mlp_forward(q, np.array([[-1.0, 0, 0]]))[0, 0]
    assert abs(y - (10.0 - 7 / 27)) < 1e-14


# ------------------------------------------------------------------ Adam
def test_adam_first_step_closed_form():
    """From zero moments the bias-corrected moments are g and g^2, so the
    first step is -lr g / (|g| + eps) (eps = 1e-8 outside the root)."""
    rng = np.random.default_rng(3)
    g = rng.normal(size=1000) * np.logspace(-9, 1, 1000)
    lr = 3e-3
    p, m, v = oracle.adam_update(np.zeros(1000), g, np.zeros(1000), np.zeros(1000), lr, 1)
    np.testing.assert_allclose(p, -lr * g / (np.abs(g) + 1e-8), rtol=1e-13)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14)
    # |g| = eps: exactly half a step
    p, _, _ = oracle.adam_update([0.0], [1e-8], [0.0], [0.0], lr, 1)
    np.testing.assert_allclose(p, [-lr / 2], rtol=1e-12)


def test_adam_constant_gradient():
    """With a constant gradient the corrected moments stay g and g^2 at every
    step (m_t = (1 - beta1^t) g, v_t = (1 - beta2^t) g^2), so each step moves
    by -lr g / (|g| + eps)."""
    g = np.array([2.0, -0.5, 1e-3, -7.0])
    p0 = np.array([0.1, 0.2, 0.3, 0.4])
    p, m, v = p0.copy(), np.zeros(4), np.zeros(4)
    lr = 1e-2
    for step in range(1, 51):
        p, m, v = oracle.adam_update(p, g, m, v, lr, step)
        np.testing.assert_allclose(m, (1 - 0.9 ** step) * g, rtol=1e-13)
        np.testing.assert_allclose(v, (1 - 0.999 ** step) * g * g, rtol=1e-12)
    np.testing.assert_allclose(p - p0, -50 * lr * g / (np.abs(g) + 1e-8), rtol=1e-11)


def test_adam_two_steps_by_hand():
    """g = 1 then g = -1: m_2 = 0.9 * 0.1 - 0.1 = -0.01, v_2 = 0.999 * 0.001
    + 0.001 = 0.001999; corrections 1 - 0.81 = 0.19 and 1 - 0.998001 =
    0.001999, so the second step is +lr (0.01 / 0.19) / (1 + eps)."""
    lr = 1e-3
    p, m, v = oracle.adam_update([0.0], [1.0], [0.0], [0.0], lr, 1)
    np.testing.assert_allclose(p, [-lr / (1 + 1e-8)], rtol=1e-14)
    p2, m2, v2 = oracle.adam_update(p, [-1.0], m, v, lr, 2)
    np.testing.assert_allclose(m2, [-0.01], rtol=1e-13)
    np.testing.assert_allclose(v2, [0.001999], rtol=1e-13)
    np.testing.assert_allclose(p2 - p, [lr * (0.01 / 0.19) / (1 + 1e-8)], rtol=1e-12)


def test_training_step_is_gradient_then_adam():
    rng = np.random.default_rng(8)
    p = _params(8)
    x = rng.uniform(-1, 1, (48, 3))
    t = rng.normal(size=(48, oracle.MLP_NOUT))
    m = rng.normal(size=p.size) * 1e-2
    v = rng.uniform(0, 1e-3, p.size)
    loss, p1, m1, v1 = oracle.mlp_adam(p, m, v, x, t, 2e-3, 7)
    l0, g = oracle.mlp_grad(p, x, t)
    pe, me, ve = oracle.adam_update(p, g, m, v, 2e-3, 7)
    assert loss == l0
    assert np.array_equal(p1, pe) and np.array_equal(m1, me) and np.array_equal(v1, ve)
