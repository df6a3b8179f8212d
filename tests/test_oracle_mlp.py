"""Pins for the band-model reference (features, bf16 rounding, gradients, Adam)."""
from collections import Counter

import numpy as np
import torch

from oracle import mlp


def test_kmer_counts_brute_force():
    rng = np.random.default_rng(0)
    for L in [0, 3, 4, 5, 50, 300]:
        s = rng.integers(0, 4, L)
        ref = Counter(tuple(s[i:i + 4]) for i in range(L - 3))
        c = mlp.kmer_counts(s)
        assert c.sum() == max(L - 3, 0)
        for kmer, cnt in ref.items():
            idx = kmer[0] * 64 + kmer[1] * 16 + kmer[2] * 4 + kmer[3]
            assert c[idx] == cnt


def test_features_layout():
    a = np.array([0, 1, 2, 3, 0], np.uint8)
    b = np.array([0, 1, 2, 3], np.uint8)
    x = mlp.features(a, b)
    assert x.shape == (259,)
    assert np.isclose(x[0], 5 / 20000) and np.isclose(x[1], 4 / 20000) and np.isclose(x[2], 1 / 20000)
    # a has ACGT and CGTA, b has ACGT: difference only at CGTA = 1*64+2*16+3*4+0
    d = np.zeros(256)
    d[1 * 64 + 2 * 16 + 3 * 4 + 0] = 1 / 5
    assert np.allclose(x[3:], d)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(size=10000) * 10.0 ** rng.integers(-8, 8, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.0078125, 3.4e38, -1e-40]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    p = mlp.init_params(3).astype(np.float64)
    p[mlp.H1 * mlp.D_IN: mlp.H1 * mlp.D_IN + mlp.H1] = rng.normal(size=mlp.H1) * 0.1  # b1
    X = rng.normal(size=(16, mlp.D_IN)) * 0.5
    y = rng.normal(size=16) + 2.0
    loss, g = mlp.backward(p, X, y, 0.9, quantize=False)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    for i in list(idx) + [mlp.N_PARAMS - 1]:
        h = 1e-6
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        lp = mlp.pinball(y, mlp.forward(pp, X, False)[0], 0.9)
        lm = mlp.pinball(y, mlp.forward(pm, X, False)[0], 0.9)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-4 * abs(g[i]), (i, fd, g[i])


def test_quantized_forward_uses_bf16_weights():
    p = mlp.init_params(4)
    X = np.random.default_rng(5).normal(size=(4, mlp.D_IN))
    yq, _ = mlp.forward(p, X, True)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    q = lambda W: mlp.bf16_round(W).astype(np.float64)
    h1 = np.maximum(X @ q(W1).T + b1, 0)
    h2 = np.maximum(h1 @ q(W2).T + b2, 0)
    assert np.allclose(yq, h2 @ q(w3) + b3[0], rtol=0, atol=1e-12)


def test_adam_first_step_is_signed_lr():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p, m, v = mlp.adam_step(np.zeros(4, np.float32), np.zeros(4), np.zeros(4), g, step=1, lr=0.01)
    # bias-corrected first step: m_hat = g, v_hat = g^2, so the step is lr*g/(|g|+eps)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-6, atol=1e-12)


def test_predict_width_clamps():
    w = mlp.predict_width(np.array([-1.0, 0.0, np.log1p(9.5), 50.0, np.log1p(4.2)]),
                          np.array([5, 5, 100, 7, 100]), np.array([9, 9, 90, 3, 100]),
                          np.array([0.0, 0.0, 0.0, 0.0, 1.0]))
    # 9.5 -> 10; 50 -> clamp 7; 4.2 * 2 = 8.4 -> 9
    assert w.tolist() == [0, 0, 10, 7, 9]
