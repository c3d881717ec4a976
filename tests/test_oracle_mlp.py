"""Pins of the FP64 warm-start network reference (oracle/mlp.py) against what
mathematics fixes: finite differences, a library normal CDF, least squares and
the closed form of Adam's first update."""
import numpy as np
import pytest
from scipy.stats import norm

import workloads as W
from oracle import mlp

SMALL = (5, 8, 8, 8, 6)


def test_layout_counts():
    assert mlp.n_params(W.WARM_WIDTHS) == 330_496
    p = W.mlp_init(SMALL, seed=1)
    blocks = mlp.split(p, SMALL)
    assert [b.shape for b in blocks] == [(8, 6), (8, 9), (8, 9), (6, 9)]
    assert all(np.all(b[:, -1] == 0.0) for b in blocks)


def test_gelu_is_z_times_normal_cdf():
    z = np.linspace(-8.0, 8.0, 2001)
    np.testing.assert_allclose(mlp.gelu(z), z * norm.cdf(z), rtol=1e-13, atol=1e-15)
    # gelu(-z) = gelu(z) - z (erf is odd)
    np.testing.assert_allclose(mlp.gelu(-z), mlp.gelu(z) - z, rtol=0, atol=1e-13)


def test_gelu_grad_by_differences():
    z = np.linspace(-6.0, 6.0, 241)
    h = 1e-5
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, rtol=0, atol=1e-9)
    assert mlp.gelu_grad(np.array([0.0]))[0] == pytest.approx(0.5, abs=1e-15)


def test_gradient_by_central_differences():
    p = W.mlp_init(SMALL, seed=2)
    p += np.random.default_rng(3).normal(0.0, 0.1, p.size)    # biases non-zero too
    x, t = W.mlp_batch(7, 5, 6, seed=4)
    _, g = mlp.loss_and_grad(p, SMALL, x, t)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (mlp.loss_and_grad(p + e, SMALL, x, t)[0] - mlp.loss_and_grad(p - e, SMALL, x, t)[0]) / (2 * h)
    err = np.abs(g - fd).max() / np.abs(fd).max()
    assert err <= 1e-6, err


def test_linear_net_stationary_at_least_squares():
    # no hidden layer: the loss gradient vanishes at numpy's least-squares fit
    x, t = W.mlp_batch(50, 5, 3, seed=5)
    A = np.hstack([x, np.ones((50, 1))])
    sol, *_ = np.linalg.lstsq(A, t, rcond=None)     # [6, 3]
    p = sol.T.ravel()
    loss, g = mlp.loss_and_grad(p, (5, 3), x, t)
    assert np.abs(g).max() < 1e-12
    assert loss == pytest.approx(np.mean((A @ sol - t) ** 2), rel=1e-12)
    # and a step away from it has a non-zero gradient pointing back
    q = p + 0.01
    _, g2 = mlp.loss_and_grad(q, (5, 3), x, t)
    assert np.dot(g2, q - p) > 0


def test_adam_first_update_closed_form():
    # at the first update m_hat = g and v_hat = g^2, so w moves by lr g / (|g| + eps)
    g = np.array([3.0, -0.5, 1e-3, 0.0, -7.0])
    w0 = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    opt = mlp.Adam(5, lr=0.01, eps=1e-8)
    w1 = opt.step(w0, g)
    np.testing.assert_allclose(w1, w0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-15, atol=1e-15)


def test_training_reduces_loss():
    p = W.mlp_init(SMALL, seed=6)
    x, _ = W.mlp_batch(64, 5, 6, seed=7)
    t = np.sin(x[:, :1]) * np.arange(1, 7) / 6.0        # a smooth target
    w, hist = mlp.train(p, SMALL, x, t, steps=300, lr=3e-3)
    assert hist[-1] < 0.1 * hist[0]
