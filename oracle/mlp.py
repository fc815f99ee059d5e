"""Plain FP64 reference of the plan selector's latency network.

TEST INFRASTRUCTURE ONLY: imported by the tests, never by the library.

The network is a 3-layer perceptron with ReLU hidden layers,
    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = w3 . h2 + b3,
trained on the mean squared error (1/B) sum_b (y_b - t_b)^2 with Adam
(Kingma & Ba 2015).  The parameter vector is laid out
W1[H][F], b1[H], W2[H][H], b2[H], w3[H], b3 -- the same flat order the
library uses, so a vector read from the device can be passed here as is.
Gradients follow from the chain rule, written out layer by layer; the
tests pin them to central finite differences, not to this code.
"""
from __future__ import annotations

import numpy as np


def n_params(F: int, H: int) -> int:
    return H * F + H + H * H + H + H + 1


def unpack(p: np.ndarray, F: int, H: int):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * F].reshape(H, F); o += H * F
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    w3 = p[o:o + H]; o += H
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3) -> np.ndarray:
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]]).astype(np.float64)


def forward(p, F: int, H: int, x: np.ndarray) -> np.ndarray:
    W1, b1, W2, b2, w3, b3 = unpack(p, F, H)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.maximum(x @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ w3 + b3


def loss(p, F: int, H: int, x, t) -> float:
    r = forward(p, F, H, x) - np.asarray(t, dtype=np.float64)
    return float(np.mean(r * r))


def grad(p, F: int, H: int, x, t):
    """Gradient of the mean squared error and the loss itself."""
    W1, b1, W2, b2, w3, b3 = unpack(p, F, H)
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    B = x.shape[0]
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    r = y - t
    dy = 2.0 * r / B                       # dL/dy_b
    g_b3 = dy.sum()
    g_w3 = h2.T @ dy
    d2 = np.outer(dy, w3) * (z2 > 0)       # dL/dz2
    g_b2 = d2.sum(axis=0)
    g_W2 = d2.T @ h1
    d1 = (d2 @ W2) * (z1 > 0)              # dL/dz1
    g_b1 = d1.sum(axis=0)
    g_W1 = d1.T @ x
    return pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3), float(np.mean(r * r))


def adam_step(p, m, v, g, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; step counts from 1.  Returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
