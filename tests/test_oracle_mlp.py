"""Pins of the cost-model network oracle: central finite differences of its
own loss (an independent route to every gradient entry) and a closed form."""
import numpy as np

from oracle import mlp


def _problem(D=5, n=40, seed=3):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, 0.3, mlp.param_count(D))
    X = rng.normal(0.0, 1.0, (n, D))
    t = rng.normal(0.0, 1.0, n)
    return p, X, t, D


def test_gradient_matches_finite_differences():
    p, X, t, D = _problem()
    g = mlp.grad(p, X, t, D)
    h = 1e-6
    rng = np.random.default_rng(0)
    # every bias, output weight and a sample of each weight matrix
    idx = list(range(mlp.H * D, mlp.H * D + mlp.H))
    idx += list(rng.choice(mlp.H * D, 40, replace=False))
    o2 = mlp.H * D + mlp.H
    idx += list(o2 + rng.choice(mlp.H * mlp.H, 60, replace=False))
    idx += list(range(o2 + mlp.H * mlp.H, mlp.param_count(D)))
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (mlp.loss(p + e, X, t, D) - mlp.loss(p - e, X, t, D)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), k


def test_constant_network_closed_form():
    """All weights zero: y = b3 for every sample, so the loss is
    mean((b3 - t)^2) and its gradient is 2 mean(b3 - t) for b3, zero for
    everything else (ReLU units are off)."""
    D = 4
    p = np.zeros(mlp.param_count(D))
    p[-1] = 0.7
    t = np.array([0.1, -0.3, 2.0])
    X = np.ones((3, D))
    assert np.allclose(mlp.forward(p, X, D), 0.7)
    g = mlp.grad(p, X, t, D)
    assert abs(g[-1] - 2 * np.mean(0.7 - t)) < 1e-15
    assert not np.any(g[:-1])


def test_planted_mistake_is_caught():
    """A gradient with the ReLU mask dropped fails the finite-difference pin."""
    p, X, t, D = _problem(seed=5)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p, D)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    dy = 2.0 * (y - t) / X.shape[0]
    wrong_db2 = np.outer(dy, w3).sum(axis=0)          # mask (z2 > 0) dropped
    k0 = mlp.H * D + mlp.H + mlp.H * mlp.H
    h = 1e-6
    bad = 0
    for j in range(mlp.H):
        e = np.zeros_like(p)
        e[k0 + j] = h
        fd = (mlp.loss(p + e, X, t, D) - mlp.loss(p - e, X, t, D)) / (2 * h)
        bad += abs(fd - wrong_db2[j]) > 1e-6 * max(1.0, abs(fd))
    assert bad > 0
