"""Band-width model reference: k-mer features and a small MLP (FP64).

TEST INFRASTRUCTURE ONLY.

The band certificate (``oracle.band``) accepts any half-width w >= w_cert;
the model predicts w_cert from cheap pair features so that most pairs
certify on the first banded pass.  It can only change speed, never results.

Features (259 per pair), following the band-model design:
  * m / 20000, n / 20000, (m - n) / 20000;
  * for each of the 256 overlapping 4-mers (index sum_t c_t * 4**(3-t), first
    base most significant): (count in a - count in b) / max(m, n).
Network: 259 -> 64 (ReLU) -> 64 (ReLU) -> 1, weights rounded to bfloat16
(round to nearest even) for the forward and backward passes, everything
else in float (here float64).
Loss: pinball (quantile) loss with tau, on the target log1p(w_cert),
averaged over the batch; the subgradient at zero residual uses the tau branch.
Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
float32 master weights.

Parameter layout (one flat vector, this order): W1 [64][259] (row = hidden
unit), b1 [64], W2 [64][64], b2 [64], w3 [64], b3 [1].
"""
from __future__ import annotations

import numpy as np

D_IN, H1, H2 = 259, 64, 64
KMER = 4
N_PARAMS = H1 * D_IN + H1 + H2 * H1 + H2 + H2 + 1
LEN_SCALE = 20000.0


def kmer_counts(seq) -> np.ndarray:
    """Counts of the overlapping 4-mers of a code sequence (256 bins)."""
    s = np.asarray(seq, dtype=np.int64)
    out = np.zeros(256, np.int64)
    if s.shape[0] < KMER:
        return out
    idx = s[:-3] * 64 + s[1:-2] * 16 + s[2:-1] * 4 + s[3:]
    np.add.at(out, idx, 1)
    return out


def features(a, b) -> np.ndarray:
    m, n = len(a), len(b)
    x = np.zeros(D_IN, np.float64)
    x[0] = m / LEN_SCALE
    x[1] = n / LEN_SCALE
    x[2] = (m - n) / LEN_SCALE
    denom = float(max(m, n, 1))
    x[3:] = (kmer_counts(a) - kmer_counts(b)) / denom
    return x


def bf16_round(x) -> np.ndarray:
    """float32 -> bfloat16 -> float32 with round-to-nearest-even."""
    f = np.asarray(x, dtype=np.float32).copy()
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    nan = np.isnan(f)
    out = u.astype(np.uint32).view(np.float32)
    out[nan] = np.float32("nan")
    return out


def unpack(params):
    p = np.asarray(params)
    o = 0
    W1 = p[o:o + H1 * D_IN].reshape(H1, D_IN); o += H1 * D_IN
    b1 = p[o:o + H1]; o += H1
    W2 = p[o:o + H2 * H1].reshape(H2, H1); o += H2 * H1
    b2 = p[o:o + H2]; o += H2
    w3 = p[o:o + H2]; o += H2
    b3 = p[o:o + 1]; o += 1
    assert o == N_PARAMS
    return W1, b1, W2, b2, w3, b3


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (float32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in [(D_IN, H1), (H1, H2)]:
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    parts.append(rng.uniform(-np.sqrt(6.0 / H2), np.sqrt(6.0 / H2), size=H2))
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float32)


def forward(params, X, quantize=True):
    """Returns (yhat, cache).  Weights are the bfloat16 rounding of params
    (quantize=False uses them as given, for finite-difference checks)."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    q = bf16_round if quantize else (lambda W: W)
    qW1, qW2, qw3 = (np.asarray(q(W), np.float64) for W in (W1, W2, w3))
    X = np.asarray(X, np.float64)
    Z1 = X @ qW1.T + b1.astype(np.float64)
    A1 = np.maximum(Z1, 0.0)
    Z2 = A1 @ qW2.T + b2.astype(np.float64)
    A2 = np.maximum(Z2, 0.0)
    y = A2 @ qw3 + float(b3[0])
    return y, (X, Z1, A1, Z2, A2, qW2, qw3)


def pinball(y, yhat, tau):
    u = np.asarray(y, np.float64) - yhat
    return float(np.mean(np.where(u < 0, (tau - 1.0) * u, tau * u)))


def backward(params, X, y, tau, quantize=True):
    """Loss and gradient w.r.t. the flat parameters (through the bf16 weights,
    i.e. the straight-through gradient of the rounding)."""
    yhat, (X, Z1, A1, Z2, A2, qW2, qw3) = forward(params, X, quantize)
    B = X.shape[0]
    u = np.asarray(y, np.float64) - yhat
    loss = float(np.mean(np.where(u < 0, (tau - 1.0) * u, tau * u)))
    dy = -np.where(u < 0, tau - 1.0, tau) / B
    dw3 = A2.T @ dy
    db3 = np.array([dy.sum()])
    dA2 = np.outer(dy, qw3)
    dZ2 = dA2 * (Z2 > 0)
    dW2 = dZ2.T @ A1
    db2 = dZ2.sum(0)
    dA1 = dZ2 @ qW2
    dZ1 = dA1 * (Z1 > 0)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(0)
    grad = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, db3])
    return loss, grad


def adam_step(params, m, v, grad, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (float64 arithmetic on float32 state); returns new (params, m, v)."""
    p = np.asarray(params, np.float64)
    g = np.asarray(grad, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    p = p - lr * mh / (np.sqrt(vh) + eps)
    return p.astype(np.float32), m.astype(np.float32), v.astype(np.float32)


def predict_width(yhat, m, n, margin):
    """Half-width from a prediction of log1p(w): ceil(expm1(yhat) * (1 + margin)),
    clamped to [0, max(m, n)]."""
    w = np.ceil(np.expm1(np.maximum(yhat, 0.0)) * (1.0 + margin))
    return np.clip(w, 0, np.maximum(m, n)).astype(np.int64)
