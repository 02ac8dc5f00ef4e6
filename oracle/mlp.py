"""CPU reference of the learned row-size predictor -- TEST INFRASTRUCTURE ONLY.

The predictor is not part of the paper; it stands in for the allocation step
of Section II-B (the upper-bound and precise allocation methods) with a size
estimate learned from the precise method's own symbolic counts.  This module
computes, in float64 and with plain numpy, everything the GPU kernels of the
learned path compute, so that the kernels can be checked:

  raw_features        the 6 per-row features (counts relative to B's columns)
  forward(params, x)  a 6 -> 64 -> 64 -> 1 perceptron with ReLU
  loss_and_grad       mean squared error and its analytic gradient
  adam_step           one step of Adam (Kingma & Ba, ICLR 2015, Algorithm 1)
  predict_sizes       predicted row sizes from the network output

Parameter layout (a flat float vector of 4673 entries), shared with the GPU
library only as a documented format:
  W1[6][64], b1[64], W2[64][64], b2[64], W3[64], b3[1]   (row-major, in this order)
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 6, 64
SIZES = [("W1", (N_IN, N_H)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("W3", (N_H,)),
         ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)  # 4673


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in SIZES])


def init_params(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, float32 values."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {
        "W1": rng.standard_normal((N_IN, N_H)) * np.sqrt(2.0 / N_IN),
        "b1": np.zeros(N_H),
        "W2": rng.standard_normal((N_H, N_H)) * np.sqrt(2.0 / N_H),
        "b2": np.zeros(N_H),
        "W3": rng.standard_normal(N_H) * np.sqrt(2.0 / N_H),
        "b3": np.zeros(1),
    }
    return pack(p).astype(np.float32)


def raw_features(nnza, nprod, maxb, minb, span, ncols):
    """The 6 features of a row of C = A*B: log1p of the list count,
    log((1 + product count) / N), log1p of the longest and shortest list,
    log(column span / N) and log1p(nprod / span), with N = max(1, B's column
    count) and a span of 0 taken as 1.  The product count and the span enter
    relative to the column space, so that rows of matrices of different sizes
    with the same density of collisions look alike."""
    nnza, nprod, maxb, minb, span = (np.asarray(a, np.float64) for a in (nnza, nprod, maxb, minb, span))
    n = float(max(int(ncols), 1))
    ratio = np.where(span > 0, nprod / np.maximum(span, 1.0), 0.0)
    return np.stack([np.log1p(nnza), np.log((1.0 + nprod) / n), np.log1p(maxb), np.log1p(minb),
                     np.log(np.maximum(span, 1.0) / n), np.log1p(ratio)], axis=1)


def forward(theta, x):
    """x: (n, 6) normalised features.  Returns (y_hat, cache)."""
    p = unpack(np.asarray(theta, np.float64))
    z1 = x @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"] + p["b3"][0]
    return y, (x, z1, h1, z2, h2, p)


def loss_and_grad(theta, x, t):
    """Mean squared error over the batch and its gradient (backpropagation
    through the two ReLU layers)."""
    y, (x, z1, h1, z2, h2, p) = forward(theta, x)
    n = x.shape[0]
    d = y - t
    loss = float(np.mean(d * d))
    dy = 2.0 * d / n
    g = {"W3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dh2 = np.outer(dy, p["W3"]) * (z2 > 0)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ p["W2"].T) * (z1 > 0)
    g["W1"] = x.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return loss, pack(g)


def adam_step(theta, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam, step number t >= 1: returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def predict_sizes(y_hat, delta, nprod, lo, hi):
    """Row size estimate ceil(nprod * exp(y_hat + delta)) clamped to the exact
    bounds [lo, hi] of the row."""
    s = np.ceil(np.asarray(nprod, np.float64) * np.exp(np.asarray(y_hat, np.float64) + delta))
    return np.clip(s, lo, hi).astype(np.int64)
