"""ORACLE (test infrastructure): the planner's cost-model network in FP64.

The network is the learned part of the planner: features of a candidate
plan in, predicted log run time out.  Architecture: 5 -> 64 -> 64 -> 1,
ReLU after the two hidden layers, mean-squared-error loss, Adam.

Conventions shared with the GPU kernels (stated, not shared code):
  X is (B, 5) row-major; a layer is h = act(x W + b) with W stored
  (fan_in, fan_out) row-major.  The flat parameter vector is
  [W1 (5*64), b1 (64), W2 (64*64), b2 (64), W3 (64*1), b3 (1)], 4609 values.
  Loss L = (1/B) sum_i (y_i - t_i)^2.
  Adam (Kingma and Ba, ICLR 2015) with bias correction:
    m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2
    p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
"""
from __future__ import annotations

import numpy as np

D_IN, H1, H2, D_OUT = 5, 64, 64, 1
SHAPES = [("W1", (D_IN, H1)), ("b1", (H1,)), ("W2", (H1, H2)), ("b2", (H2,)),
          ("W3", (H2, D_OUT)), ("b3", (D_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(flat: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + size], dtype=np.float64).reshape(shape)
        o += size
    return out


def flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel()
                           for name, _ in SHAPES])


def forward(flat: np.ndarray, X: np.ndarray):
    """Returns (y of shape (B,), cache for backward)."""
    p = unflatten(flat)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = (h2 @ p["W3"] + p["b3"])[:, 0]
    return y, (X, z1, h1, z2, h2)


def loss(y: np.ndarray, t: np.ndarray) -> float:
    d = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    return float(np.mean(d * d))


def backward(flat: np.ndarray, cache, y: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Gradient of the mean-squared loss with respect to the flat parameters
    (chain rule, written out layer by layer)."""
    p = unflatten(flat)
    X, z1, h1, z2, h2 = cache
    B = X.shape[0]
    dy = (2.0 / B) * (np.asarray(y, np.float64) - np.asarray(t, np.float64))  # (B,)
    dy = dy[:, None]
    g = {}
    g["W3"] = h2.T @ dy
    g["b3"] = dy.sum(axis=0)
    dh2 = dy @ p["W3"].T
    dz2 = dh2 * (z2 > 0.0)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"].T
    dz1 = dh1 * (z1 > 0.0)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return flatten(g)


def adam_step(flat, grad, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step counts from 1).  Returns (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return flat - lr * mhat / (np.sqrt(vhat) + eps), m, v


def numeric_grad(flat: np.ndarray, X: np.ndarray, t: np.ndarray, h: float = 1e-6) -> np.ndarray:
    """Central finite differences of the loss (a pin for ``backward``)."""
    g = np.empty_like(flat, dtype=np.float64)
    for i in range(flat.size):
        e = np.zeros_like(flat, dtype=np.float64)
        e[i] = h
        lp = loss(forward(flat + e, X)[0], t)
        lm = loss(forward(flat - e, X)[0], t)
        g[i] = (lp - lm) / (2 * h)
    return g
