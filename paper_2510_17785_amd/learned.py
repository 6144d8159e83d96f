"""Learned Chebyshev bounds: train the bound-predicting network on the GPU.

The labels are the Lanczos bounds (ln lambda_min, ln lambda_max per smoothed
level) that the library computes for a batch of independent patches; the
features are the library's patch features; training runs in the library's
forward, backward and Adam kernels.  This module only sequences those calls.
Random numbers (initial weights, sample order) are drawn here with numpy and
passed in.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from .api import BoundNet, PatchBatch, n_features

HIDDEN = 64


def glorot_params(n_in: int, n_out: int, rng: np.random.Generator) -> np.ndarray:
    """Glorot-uniform weights U(-a, a), a = sqrt(6 / (fan_in + fan_out)), zero biases,
    in the parameter layout of the library."""
    shapes = [(n_in, HIDDEN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,),
              (HIDDEN, n_out), (n_out,)]
    parts = []
    for s in shapes:
        if len(s) == 2:
            a = np.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-a, a, size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts).astype(np.float32)


@dataclasses.dataclass
class TrainResult:
    net: BoundNet
    epoch_loss: np.ndarray
    val_rmse: np.ndarray      # per output (ln lambda_min, ln lambda_max per level)
    margin: float             # 3 x the largest validation RMSE of ln lambda_max
    label_seconds: float
    train_seconds: float


def train_bound_network(dim, p, levels, vertices, coeff, epochs=40, batch=256, lr=1e-3,
                        val_frac=0.1, label_steps=30, seed=0) -> TrainResult:
    """Lanczos labels of the given random patches (pmg_patches_setup), then
    pmg_mlp_fit_bounds: features, ln-bound targets, standardiser, training,
    validation and margin in the library.  This function draws the random
    numbers (initial weights, the validation split, the sample order of every
    epoch) and sequences the calls."""
    import time
    n = vertices.shape[0]
    t0 = time.perf_counter()
    lab = PatchBatch(dim, p, vertices, coeff, levels=levels, precision="fp64",
                     lanczos_steps=label_steps, seed=seed)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_out = 2 * (len(levels) - 1)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    n_val = max(1, int(val_frac * n))
    val, tr = perm[:n_val], perm[n_val:]
    net = BoundNet(n_features(dim), n_out, glorot_params(n_features(dim), n_out, rng),
                   max_batch=max(batch, 1024, n_val))
    order = np.stack([tr[rng.permutation(len(tr))] for _ in range(epochs)]).astype(np.int32)
    hist, rmse, margin = net.fit_bounds(lab, torch.tensor(order, device="cuda"),
                                        torch.tensor(val.astype(np.int32), device="cuda"),
                                        epochs, batch, lr)
    lab.close()
    t2 = time.perf_counter()
    return TrainResult(net, hist, rmse, margin, t1 - t0, t2 - t1)
