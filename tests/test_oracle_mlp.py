"""Pins of the float64 MLP oracle: finite differences, closed forms, Adam's first step."""
import numpy as np
import pytest

from oracle import mlp


def test_parameter_count():
    assert mlp.n_params() == 4866


def test_forward_closed_form():
    """Zero weights: the output is the last bias; a single active path is a product of weights."""
    th = np.zeros(mlp.n_params())
    p = mlp.unpack(th)
    p["b3"][:] = [1.5, -2.0]
    X = np.random.default_rng(0).normal(size=(4, 8))
    y, _ = mlp.forward(th, X)
    assert np.array_equal(y, np.tile([1.5, -2.0], (4, 1)))
    # one path: x0 -> h1[3] -> h2[5] -> y[1]
    p["b3"][:] = 0.0
    p["W1"][3, 0] = 2.0
    p["W2"][5, 3] = 3.0
    p["W3"][1, 5] = -0.5
    X = np.array([[1.0] + [0.0] * 7, [-1.0] + [0.0] * 7])
    y, _ = mlp.forward(th, X)
    assert np.array_equal(y, np.array([[0.0, -3.0], [0.0, 0.0]]))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    th = mlp.init(seed)
    th[np.isin(np.arange(th.size), np.arange(512, 576))] = rng.normal(size=64) * 0.1  # nonzero b1
    X = rng.normal(size=(7, 8))
    Y = rng.normal(size=(7, 2))
    L, g = mlp.loss_grad(th, X, Y)
    assert np.isclose(L, mlp.loss(th, X, Y), rtol=1e-15)
    idx = np.concatenate([rng.choice(th.size, 300, replace=False), np.arange(th.size - 2, th.size)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (mlp.loss(th + e, X, Y) - mlp.loss(th - e, X, Y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8


def test_adam_first_step_closed_form():
    """After one step from m = v = 0, Adam moves each parameter by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    th1, m, v = mlp.adam_step(th, g, np.zeros(50), np.zeros(50), 1, lr=1e-2)
    assert np.allclose(th1, th - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    rng = np.random.default_rng(4)
    X = rng.normal(size=(64, 8))
    Y = np.stack([np.tanh(X[:, 0] - X[:, 1]), 0.5 * X[:, 2]], axis=1)
    th = mlp.init(0)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    L0 = mlp.loss(th, X, Y)
    for t in range(1, 301):
        L, g = mlp.loss_grad(th, X, Y)
        th, m, v = mlp.adam_step(th, g, m, v, t, lr=3e-3)
    assert mlp.loss(th, X, Y) < 0.1 * L0


def test_standardise_guards_zero_variance():
    F = np.array([[1.0, 0.0, 5.0], [3.0, 0.0, 5.0]])
    mu, sd = mlp.standardise_fit(F)
    assert np.array_equal(mu, [2.0, 0.0, 5.0]) and np.array_equal(sd, [1.0, 1.0, 1.0])


def test_adam_second_step_worked_value():
    """Two Adam steps on one parameter, gradients +1 then -2, lr = 0.1, worked by hand:
    step 1: m = 0.1, v = 0.001, bias-corrected 1 and 1, theta moves by -0.1;
    step 2: m = 0.9 * 0.1 - 0.2 = -0.11, v = 0.999 * 0.001 + 0.004 = 0.004999,
    m^ = -0.11 / 0.19 = -0.5789473684..., v^ = 0.004999 / 0.001999 = 2.5007503751...,
    theta moves by -0.1 m^ / sqrt(v^) = +0.0366103527035845565...
    A bias correction with the wrong power of beta, or a moment not carried over, fails."""
    th0 = np.array([0.25])
    th1, m, v = mlp.adam_step(th0, np.array([1.0]), np.zeros(1), np.zeros(1), 1, lr=0.1, eps=0.0)
    assert abs(th1[0] - 0.15) <= 1e-15
    th2, m, v = mlp.adam_step(th1, np.array([-2.0]), m, v, 2, lr=0.1, eps=0.0)
    assert abs(m[0] + 0.11) <= 1e-15 and abs(v[0] - 0.004999) <= 1e-17
    assert abs(th2[0] - (0.15 + 0.0366103527035845565282265)) <= 1e-15
