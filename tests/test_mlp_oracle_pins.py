"""Pins of the cost-model reference against calculus and closed forms."""
import numpy as np
import pytest

from oracle import mlp_ref as M


def data(n=40, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 500, (n, M.F))
    t = rng.normal(10, 1, n)
    return x, t


def test_gradient_matches_central_differences():
    x, t = data()
    p = M.init(x, t, seed=3)
    p[M.OB1:M.OW2] = 0.05  # keep pre-activations away from the ReLU kink
    L, g = M.loss_grad(p, x, t)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(np.arange(M.OW1, M.OB3 + 1), 60, replace=False),
                          [M.OB3, M.OB1, M.OB2, M.OW3]])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (M.loss(pp, x, t) - M.loss(pm, x, t)) / (2 * h)
        assert fd == pytest.approx(g[i], rel=1e-5, abs=1e-9), i
    assert np.all(g[:M.OW1] == 0) and np.all(g[M.OYM:] == 0)


def test_all_active_network_is_the_linear_map():
    """With every pre-activation positive the network is W3 (W2 (W1 u + b1)
    + b2) + b3, a closed form."""
    x, t = data(8)
    p = M.init(x, t, seed=2)
    q = M.unpack(p)
    p[M.OW1:M.OB1] = np.abs(p[M.OW1:M.OB1]) * 0.01
    p[M.OB1:M.OW2] = 10.0
    p[M.OW2:M.OB2] = np.abs(p[M.OW2:M.OB2])
    p[M.OB2:M.OW3] = 1.0
    q = M.unpack(p)
    u = (np.log1p(x) - q["xm"]) / q["xs"]
    y = q["W3"] @ (q["W2"] @ (q["W1"] @ u.T + q["b1"][:, None]) + q["b2"][:, None]) + q["b3"]
    pred, _ = M.forward(p, x)
    assert np.allclose(pred, y * q["ys"] + q["ym"], rtol=1e-13)


def test_loss_is_zero_at_the_targets_and_constant_network():
    x, t = data(10)
    p = M.init(x, t)
    p[M.OW1:M.OYM] = 0.0          # network outputs 0 in standardised units
    t_const = np.full(10, p[M.OYM])
    L, g = M.loss_grad(p, x, t_const)
    assert L == 0.0 and np.all(g == 0)


def test_first_adam_step_moves_each_weight_by_lr():
    """After one bias-corrected Adam step m_hat = g and v_hat = g^2, so every
    parameter with a nonzero gradient moves by lr * g/(|g| + eps)."""
    x, t = data()
    p = M.init(x, t, seed=5)
    _, g = M.loss_grad(p, x, t)
    lr = 1e-3
    p1 = M.adam(p, x, t, 1, lr)
    sl = slice(M.OW1, M.OB3 + 1)
    expect = p[sl] - lr * g[sl] / (np.abs(g[sl]) + 1e-8)
    assert np.allclose(p1[sl], expect, rtol=0, atol=1e-15)


def test_adam_reduces_the_loss():
    x, t = data(200)
    t = np.log1p(x[:, 0]) * 0.7 + 0.2 * np.log1p(x[:, 3])
    p = M.init(x, t, seed=1)
    L0 = M.loss(p, x, t)
    p = M.adam(p, x, t, 300, 3e-3)
    assert M.loss(p, x, t) < 0.05 * L0
