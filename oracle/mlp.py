"""FP64 reference of the sweep cost model (test infrastructure only).

The model is a fully connected network: features x (F values) -> 64 ReLU
units -> 64 ReLU units -> one output, the predicted natural log of a sweep's
run time in milliseconds.  Training minimises the mean squared error over a
data set with Adam (Kingma & Ba, ICLR 2015: m <- b1 m + (1-b1) g,
v <- b2 v + (1-b2) g^2, p <- p - lr * m_hat / (sqrt(v_hat) + eps) with
bias-corrected m_hat, v_hat).

Parameter vector layout (shared with the library only as a documented format):
W1 (H x F, row-major), b1 (H), W2 (H x H), b2 (H), w3 (H), b3 (1).

Pinned in tests/test_oracle_mlp.py by central finite differences and by a
least-squares closed form for the output layer.
"""
from __future__ import annotations

import numpy as np

F = 16
H = 64


def num_params(f: int = F, h: int = H) -> int:
    return h * f + h + h * h + h + h + 1


def unpack(p: np.ndarray, f: int = F, h: int = H):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + h * f].reshape(h, f)
    o += h * f
    b1 = p[o:o + h]
    o += h
    W2 = p[o:o + h * h].reshape(h, h)
    o += h * h
    b2 = p[o:o + h]
    o += h
    w3 = p[o:o + h]
    o += h
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def forward(p: np.ndarray, X: np.ndarray) -> np.ndarray:
    W1, b1, W2, b2, w3, b3 = unpack(p, X.shape[1])
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ w3 + b3


def loss(p: np.ndarray, X: np.ndarray, y: np.ndarray) -> float:
    r = forward(p, X) - y
    return float(np.mean(r * r))


def grad(p: np.ndarray, X: np.ndarray, y: np.ndarray):
    """Loss and its gradient by reverse-mode differentiation of the layers."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n, f = X.shape
    W1, b1, W2, b2, w3, b3 = unpack(p, f)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    out = h2 @ w3 + b3
    r = out - y
    L = float(np.mean(r * r))
    dout = 2.0 * r / n
    gw3 = h2.T @ dout
    gb3 = np.sum(dout)
    dh2 = np.outer(dout, w3) * (a2 > 0)
    gW2 = dh2.T @ h1
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2) * (a1 > 0)
    gW1 = dh1.T @ X
    gb1 = dh1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, [gb3]])
    return L, g


def adam_step(p, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
