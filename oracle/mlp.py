"""CPU FP64 oracle for the cost model's network.

TEST INFRASTRUCTURE ONLY: imported by the test suite, never by the library.
Plain numpy in float64, one definition per formula, no blocking: the
network is fully connected with two hidden layers of H ReLU units and a
linear output,

    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = w3 . h2 + b3,

its loss over n samples is the mean squared error (1/n) sum (y - t)^2, and
the gradient follows the chain rule one factor at a time.  Parameters use
the flat layout of the library's network (W1 [H][D] row-major, b1, W2
[H][H], b2, w3, b3).  The network is not from the Sympiler paper (which
tunes variant thresholds by hand); it is this project's cost model, pinned
here against central finite differences and a closed form.
"""
from __future__ import annotations

import numpy as np

H = 64


def param_count(D: int) -> int:
    return H * D + H + H * H + H + H + 1


def unpack(p, D: int):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * D].reshape(H, D); o += H * D
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def forward(p, X, D: int):
    """Outputs y (n,) for samples X (n, D)."""
    W1, b1, W2, b2, w3, b3 = unpack(p, D)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ w3 + b3


def loss(p, X, t, D: int) -> float:
    y = forward(p, X, D)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grad(p, X, t, D: int) -> np.ndarray:
    """Gradient of the mean squared error, flat like the parameters."""
    W1, b1, W2, b2, w3, b3 = unpack(p, D)
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    n = X.shape[0]
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    dy = 2.0 * (y - t) / n                      # dL/dy
    dw3 = h2.T @ dy
    db3 = dy.sum()
    dz2 = np.outer(dy, w3) * (z2 > 0)           # dL/dz2
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)                 # dL/dz1
    dW1 = dz1.T @ X
    db1 = dz1.sum(axis=0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, [db3]])
