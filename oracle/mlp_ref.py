"""Reference of the run-time model: a two-hidden-layer perceptron trained by
Adam on the mean squared error, in float64 NumPy.

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU baseline).

    h1 = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = W3 h2 + b3,
    loss = mean over rows of (y - t)^2.

Parameters are passed in and returned as a dict of arrays
{W1 (H x F), b1 (H), W2 (H x H), b2 (H), W3 (1 x H), b3 (1)}; the flat
order used by the GPU library is W1, b1, W2, b2, W3, b3, each row-major.
Adam: m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def flatten(P) -> np.ndarray:
    return np.concatenate([np.asarray(P[k], dtype=np.float64).ravel() for k in ORDER])


def unflatten(v: np.ndarray, F: int, H: int):
    shapes = {"W1": (H, F), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (1, H), "b3": (1,)}
    out, o = {}, 0
    for k in ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = np.asarray(v[o:o + n], dtype=np.float64).reshape(shapes[k])
        o += n
    return out


def forward(P, X):
    z1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ P["W3"].T + P["b3"]
    return y[:, 0], (X, z1, h1, z2, h2)


def loss_and_grads(P, X, t):
    y, (X, z1, h1, z2, h2) = forward(P, X)
    R = X.shape[0]
    loss = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / R                    # d loss / d y
    g = {"W3": dy[None, :] @ h2, "b3": np.array([dy.sum()])}
    dh2 = dy[:, None] * P["W3"][0][None, :]
    dz2 = dh2 * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ P["W2"]
    dz1 = dh1 * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return loss, g


def adam_train(P, X, t, epochs: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999,
               eps: float = 1e-8):
    """Full-batch Adam; returns the trained parameters and the loss per epoch
    (before each update)."""
    P = {k: np.array(v, dtype=np.float64) for k, v in P.items()}
    m = {k: np.zeros_like(v) for k, v in P.items()}
    v = {k: np.zeros_like(x) for k, x in P.items()}
    losses = []
    for step in range(1, epochs + 1):
        loss, g = loss_and_grads(P, X, t)
        losses.append(loss)
        for k in ORDER:
            m[k] = b1 * m[k] + (1 - b1) * g[k]
            v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
            mh = m[k] / (1 - b1 ** step)
            vh = v[k] / (1 - b2 ** step)
            P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return P, losses
