"""Training of the learned row-size predictor from the method's own symbolic
counts.  Features, targets, normalisation statistics, forward and backward
passes and Adam run in the library's HIP kernels; for the safety margin the
network's outputs come from the forward kernel and spg_mlp_calibrate takes the
residuals and their quantile on the host (one selection).  This module only gathers
the rows, shuffles them and calls the entry points in order."""
from __future__ import annotations

import numpy as np
import torch

from . import ALLOC_PRECISE, OPT_ALLOC, DeviceCSR, Handle


def he_init(seed: int) -> np.ndarray:
    """Initial parameters: He-normal weights (std sqrt(2 / fan_in)) drawn from
    PCG64(seed) in the order W1, W2, W3; zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w1 = rng.standard_normal((6, 64)) * np.sqrt(2.0 / 6)
    w2 = rng.standard_normal((64, 64)) * np.sqrt(2.0 / 64)
    w3 = rng.standard_normal(64) * np.sqrt(2.0 / 64)
    return np.concatenate([w1.ravel(), np.zeros(64), w2.ravel(), np.zeros(64), w3, np.zeros(1)]).astype(np.float32)


def collect(h: Handle, pairs):
    """Features and targets (log of nnz(C_i) / nprod_i) of every predicted row
    of each product A*B, from a precise symbolic pass."""
    old = h.get_option(OPT_ALLOC)
    h.set_option(OPT_ALLOC, ALLOC_PRECISE)
    fs, ts = [], []
    try:
        for A, B in pairs:
            c_rpt, _ = h.symbolic(A, B)
            feats, targets, pred, _, _ = h.mlp_features(A, B, c_rpt)
            keep = pred.bool()
            fs.append(feats[keep])
            ts.append(targets[keep])
    finally:
        h.set_option(OPT_ALLOC, old)
    return torch.cat(fs), torch.cat(ts)


def train(h: Handle, feats: torch.Tensor, targets: torch.Tensor, seed: int = 0, epochs: int = 8,
          batch: int = 4096, lr: float = 1e-3, quantile: float = 0.99):
    """Initialise, fit the normalisation, train with Adam on shuffled rows
    (equal weight per source is the caller's choice of rows) and calibrate the
    margin.  Returns (loss before, loss after, delta)."""
    h.mlp_set_params(he_init(seed), np.array([0.0] * 6 + [1.0] * 6, np.float32), 0.0)
    h.mlp_fit_normalization(feats)
    loss0 = h.mlp_loss(feats, targets)
    g = torch.Generator().manual_seed(seed)
    for _ in range(epochs):
        perm = torch.randperm(feats.shape[0], generator=g).to(feats.device)
        h.mlp_train(feats[perm], targets[perm], 1, batch, lr)
    loss1 = h.mlp_loss(feats, targets)
    delta = h.mlp_calibrate(feats, targets, quantile)
    return loss0, loss1, delta
