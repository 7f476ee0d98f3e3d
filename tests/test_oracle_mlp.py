"""Pins of the rank-predictor oracle (oracle/mlp.py) on the CPU: the analytic
gradient against central finite differences, closed forms of the loss and
of its gradient for a network whose last layer is zero, the asymmetry of the
loss, the first Adam step, the parameter count and the box features."""

import numpy as np

from oracle import mlp


def _data(n=40, seed=1):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 6))
    rank = rng.integers(5, 120, n).astype(np.float64)
    return x, rank


def test_parameter_count():
    assert mlp.n_params() == 8833


def test_gradient_matches_finite_differences():
    x, rank = _data()
    p = mlp.init_params(3) * 0.5
    p[:] += 0.01  # positive biases keep ReLUs active away from kinks
    L, g = mlp.loss_and_grad(p, x, rank, alpha=4.0)
    rng = np.random.default_rng(7)
    idx = rng.choice(p.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        Lp, _ = mlp.loss_and_grad(p + e, x, rank, 4.0)
        Lm, _ = mlp.loss_and_grad(p - e, x, rank, 4.0)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_zero_last_layer_closed_form():
    x, rank = _data()
    p = mlp.init_params(5)
    W4 = slice(mlp.n_params() - 65, mlp.n_params() - 1)
    p[W4] = 0.0
    p[-1] = 3.0  # yhat = b4 = 3 for every sample
    alpha = 2.5
    L, g = mlp.loss_and_grad(p, x, rank, alpha)
    r = 3.0 - np.log(rank)
    c = np.where(r < 0, alpha, 1.0)
    assert abs(L - np.mean(c * r * r)) < 1e-12
    assert abs(g[-1] - np.mean(2 * c * r)) < 1e-12
    # the hidden layers receive no gradient through a zero last layer
    assert np.all(g[:mlp.n_params() - 65] == 0.0)


def test_loss_asymmetry():
    x, rank = _data()
    p = mlp.init_params(2)
    p[mlp.n_params() - 65:mlp.n_params() - 1] = 0.0
    p[-1] = 10.0  # over-predicts every sample: alpha has no effect
    assert mlp.loss_and_grad(p, x, rank, 1.0)[0] == mlp.loss_and_grad(p, x, rank, 9.0)[0]
    p[-1] = 0.0  # under-predicts every sample: the loss scales with alpha
    L1 = mlp.loss_and_grad(p, x, rank, 1.0)[0]
    L9 = mlp.loss_and_grad(p, x, rank, 9.0)[0]
    assert abs(L9 - 9.0 * L1) < 1e-12 * L9


def test_first_adam_step_is_signed_lr():
    g = np.array([0.3, -2.0, 1e-3])
    p0 = np.zeros(3)
    p1, m, v = mlp.adam_step(p0, g, np.zeros(3), np.zeros(3), t=1, lr=0.01, eps=0.0)
    assert np.allclose(p1, -0.01 * np.sign(g), rtol=0, atol=1e-15)


def test_box_features_circle():
    n = 256
    th = 2 * np.pi * np.arange(n) / n
    x = np.stack([np.cos(th), np.sin(th)], axis=1)
    kappa = np.ones(n)
    f = mlp.box_features(x, kappa, 0, n, 10.0, 15.0, 0, 1e-10)
    # the whole unit circle: diameter 2, unit curvature
    assert abs(f[0] - 20.0) < 1e-12 and abs(f[1] - 30.0) < 1e-12
    assert abs(f[2] - 2.0) < 1e-12 and abs(f[3] - 2.0) < 1e-12
    assert f[4] == 0.0 and abs(f[5] + 10.0) < 1e-12
