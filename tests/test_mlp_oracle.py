"""Pins of the reference MLP (the gradient oracle for the GPU cost model)."""
import numpy as np
import pytest

from oracle import mlp


@pytest.mark.parametrize("shape,seed", [((5, 7, 3), 0), ((14, 32, 32), 1), ((1, 1, 1), 2)])
def test_gradient_matches_central_differences(shape, seed):
    n_in, h1, h2 = shape
    rng = np.random.default_rng(seed)
    p = mlp.init(n_in, h1, h2, seed) + 0.1 * rng.normal(size=mlp.param_count(n_in, h1, h2))
    X = rng.normal(size=(9, n_in))
    t = rng.normal(size=9)
    g = mlp.grad(p, X, t, n_in, h1, h2)
    gn = mlp.numeric_grad(p, X, t, n_in, h1, h2)
    assert np.abs(g - gn).max() <= 1e-7 * max(1.0, np.abs(gn).max())


def test_forward_special_cases():
    # all weights zero except the output bias: the network is a constant
    n_in, h1, h2 = 3, 4, 2
    p = np.zeros(mlp.param_count(n_in, h1, h2))
    p[-1] = 2.5
    y, _, _ = mlp.forward(p, np.ones((5, n_in)), n_in, h1, h2)
    assert np.all(y == 2.5)
    # one path x0 -> unit 0 -> unit 0 -> y: y = tanh(tanh(x0))
    p = np.zeros(mlp.param_count(n_in, h1, h2))
    W1, b1, W2, b2, w3, _ = mlp.unpack(p, n_in, h1, h2)
    W1[0, 0] = 1.0
    W2[0, 0] = 1.0
    w3[0] = 1.0
    X = np.linspace(-2, 2, 7)[:, None] * np.eye(n_in)[0]
    y, _, _ = mlp.forward(p, X, n_in, h1, h2)
    assert np.allclose(y, np.tanh(np.tanh(X[:, 0])), rtol=0, atol=1e-15)


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.5, 1e-3])
    p1, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(p1, -0.01 * np.sign(g), rtol=0, atol=1e-15)


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    n_in, h1, h2 = 4, 16, 16
    X = rng.normal(size=(64, n_in))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]
    p = mlp.init(n_in, h1, h2, 5)
    m = np.zeros_like(p); v = np.zeros_like(p)
    l0 = mlp.loss(p, X, t, n_in, h1, h2)
    for k in range(1, 301):
        p, m, v = mlp.adam_step(p, mlp.grad(p, X, t, n_in, h1, h2), m, v, k, lr=0.01)
    assert mlp.loss(p, X, t, n_in, h1, h2) < 0.1 * l0
