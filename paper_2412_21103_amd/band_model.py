"""Training driver for the band model (host orchestration of libnw calls).

The labels come from the full-grid method itself: nw_align_batch gives each
training pair's optimal path, nw_path_labels turns it into w_path (how far
the path strays beyond the straight band, the maximum diagonal offset of the
optimal path) and the target log1p(w_path).  The band model's half-width is
the first pass of the certified band: a band that holds an optimal path
reaches the optimal score, and the certificate then widens the band straight
to the width that score certifies.  make_labels(label="cert") gives the other
label the library can train on, w_cert (from the score alone, through
nw_band_labels).  Features come from nw_mlp_features; each epoch runs in
nw_mlp_train_epoch over a seeded permutation drawn here and passed in.
"""
from __future__ import annotations

import numpy as np
import torch

from . import (PAPER_SCORING, Mlp, align_batch, band_labels, mlp_features, mlp_train_epoch,
               mlp_train_workspace_size, path_labels)


def he_uniform(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases, in the library's parameter order."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in [(259, 64), (64, 64)]:
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    parts.append(rng.uniform(-np.sqrt(6.0 / 64), np.sqrt(6.0 / 64), size=64))
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float32)


def make_labels(pool, a_off, a_len, b_off, b_len, max_len, scoring=PAPER_SCORING, label: str = "path"):
    """Full-grid results, then (scores, w, target) for every pair (device
    tensors): w = w_path from the paths (label "path") or w_cert from the
    scores (label "cert")."""
    if label == "cert":
        scores, _, _, _ = align_batch(pool, a_off, a_len, b_off, b_len, max_len, scoring, score_only=True)
        w, target = band_labels(scores, a_len, b_len, scoring)
        return scores, w, target
    if label != "path":
        raise ValueError(f"unknown label {label!r}")
    scores, paths, path_off, plen = align_batch(pool, a_off, a_len, b_off, b_len, max_len, scoring)
    w, target = path_labels(paths, path_off, plen, a_len, b_len)
    return scores, w, target


def train(x: torch.Tensor, target: torch.Tensor, epochs: int = 200, batch: int = 256,
          lr: float = 3e-3, tau: float = 0.9, seed: int = 0, init_seed: int = 0, mlp: Mlp | None = None):
    """Train on (x, target) for `epochs` passes.  Returns (mlp, per-epoch mean loss)."""
    n = int(x.shape[0])
    mlp = mlp if mlp is not None else Mlp(he_uniform(init_seed))
    rng = np.random.default_rng(seed)
    ws = torch.empty(mlp_train_workspace_size(batch), dtype=torch.uint8, device=x.device)
    history = []
    for _ in range(epochs):
        order = torch.from_numpy(rng.permutation(n).astype(np.int32)).to(x.device)
        losses = mlp_train_epoch(mlp, x, target, order, batch, tau, lr, workspace=ws)
        history.append(losses)
    torch.cuda.synchronize()
    return mlp, [float(h.mean().item()) for h in history]


def features_and_labels(pool, a_off, a_len, b_off, b_len, max_len, scoring=PAPER_SCORING, label: str = "path"):
    x = mlp_features(pool, a_off, a_len, b_off, b_len)
    scores, w, target = make_labels(pool, a_off, a_len, b_off, b_len, max_len, scoring, label)
    return x, scores, w, target
