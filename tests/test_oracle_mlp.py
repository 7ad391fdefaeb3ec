"""Pins of the FP64 cost-model reference (oracle/mlp.py)."""
import numpy as np

from oracle import mlp


def rand_params(seed, scale=0.3):
    return np.random.default_rng(seed).normal(0, scale, mlp.num_params())


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    X = rng.normal(0, 1, (37, mlp.F))
    y = rng.normal(0, 1, 37)
    p = rand_params(2)
    L, g = mlp.grad(p, X, y)
    assert abs(L - mlp.loss(p, X, y)) < 1e-14
    idx = rng.choice(p.size, 300, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, y) - mlp.loss(p - e, X, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_output_layer_gradient_vanishes_at_least_squares_optimum():
    """With the hidden layers fixed the output layer is a linear regression on
    h2; at numpy's least-squares solution the gradient w.r.t. (w3, b3) is 0."""
    rng = np.random.default_rng(3)
    X = rng.normal(0, 1, (200, mlp.F))
    y = rng.normal(0, 1, 200)
    p = rand_params(4)
    W1, b1, W2, b2, _, _ = mlp.unpack(p)
    h2 = np.maximum(np.maximum(X @ W1.T + b1, 0) @ W2.T + b2, 0)
    A = np.hstack([h2, np.ones((200, 1))])
    sol, *_ = np.linalg.lstsq(A, y, rcond=None)
    q = p.copy()
    q[-65:-1] = sol[:-1]
    q[-1] = sol[-1]
    _, g = mlp.grad(q, X, y)
    assert np.max(np.abs(g[-65:])) < 1e-10


def test_dead_units_get_no_gradient():
    p = rand_params(5)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    o = mlp.H * mlp.F
    p2 = p.copy()
    p2[o + 7] = -1e6  # b1[7]: unit 7 of layer 1 never active
    X = np.random.default_rng(6).normal(0, 1, (20, mlp.F))
    _, g = mlp.grad(p2, X, np.zeros(20))
    assert np.all(g[7 * mlp.F:(7 + 1) * mlp.F] == 0) and g[o + 7] == 0


def test_adam_first_step_is_sign_step():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, m, v = mlp.adam_step(p, np.zeros(3), np.zeros(3), g, 1, lr=0.01, eps=1e-12)
    assert np.allclose(p1, p - 0.01 * np.sign(g), atol=1e-9)


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(7)
    X = rng.uniform(-1, 1, (256, mlp.F))
    y = np.sin(X[:, 0]) + 0.5 * X[:, 1] ** 2
    p = rand_params(8, 0.2)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    L0 = mlp.loss(p, X, y)
    for t in range(1, 301):
        _, g = mlp.grad(p, X, y)
        p, m, v = mlp.adam_step(p, m, v, g, t, lr=3e-3)
    assert mlp.loss(p, X, y) < 0.1 * L0
