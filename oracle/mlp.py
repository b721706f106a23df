"""Reference MLP cost model in FP64 (test infrastructure only).

The GPU library trains and evaluates a small multilayer perceptron that
predicts the log run time of a checkpoint split from split features.  This
module is its plain definition, used to check the GPU forward pass, the GPU
gradients and the GPU optimiser step; it shares no code with the library.

Network: x (n_in) -> tanh(W1 x + b1) (h1) -> tanh(W2 a1 + b2) (h2)
-> y = w3 . a2 + b3.  Flat parameter vector, in order: W1 [h1][n_in]
row-major, b1 [h1], W2 [h2][h1], b2 [h2], w3 [h2], b3 [1].
Loss: mean over the batch of (y - target)^2.
Optimiser: Adam (Kingma & Ba 2015) with bias correction.
"""
from __future__ import annotations

import numpy as np


def param_count(n_in: int, h1: int, h2: int) -> int:
    return h1 * n_in + h1 + h2 * h1 + h2 + h2 + 1


def unpack(p: np.ndarray, n_in: int, h1: int, h2: int):
    o = 0
    W1 = p[o:o + h1 * n_in].reshape(h1, n_in); o += h1 * n_in
    b1 = p[o:o + h1]; o += h1
    W2 = p[o:o + h2 * h1].reshape(h2, h1); o += h2 * h1
    b2 = p[o:o + h2]; o += h2
    w3 = p[o:o + h2]; o += h2
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def init(n_in: int, h1: int, h2: int, seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((h1, n_in), (h2, h1)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    lim = np.sqrt(6.0 / (h2 + 1))
    parts.append(rng.uniform(-lim, lim, size=h2))
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float64)


def forward(p, X, n_in, h1, h2):
    W1, b1, W2, b2, w3, b3 = unpack(p, n_in, h1, h2)
    a1 = np.tanh(X @ W1.T + b1)
    a2 = np.tanh(a1 @ W2.T + b2)
    y = a2 @ w3 + b3
    return y, a1, a2


def loss(p, X, t, n_in, h1, h2) -> float:
    y, _, _ = forward(p, X, n_in, h1, h2)
    return float(np.mean((y - t) ** 2))


def grad(p, X, t, n_in, h1, h2):
    """Analytic gradient of the mean squared error (chain rule, layer by layer)."""
    W1, b1, W2, b2, w3, b3 = unpack(p, n_in, h1, h2)
    B = X.shape[0]
    y, a1, a2 = forward(p, X, n_in, h1, h2)
    dy = 2.0 * (y - t) / B                  # dL/dy
    g_w3 = a2.T @ dy
    g_b3 = dy.sum()
    dz2 = np.outer(dy, w3) * (1.0 - a2 ** 2)
    g_W2 = dz2.T @ a1
    g_b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - a1 ** 2)
    g_W1 = dz1.T @ X
    g_b1 = dz1.sum(axis=0)
    return np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])


def numeric_grad(p, X, t, n_in, h1, h2, eps=1e-6):
    """Central finite differences of the loss."""
    g = np.zeros_like(p)
    for i in range(len(p)):
        q = p.copy(); q[i] += eps
        lp = loss(q, X, t, n_in, h1, h2)
        q[i] -= 2 * eps
        lm = loss(q, X, t, n_in, h1, h2)
        g[i] = (lp - lm) / (2 * eps)
    return g


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at iteration `step` (1-based); returns new (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
