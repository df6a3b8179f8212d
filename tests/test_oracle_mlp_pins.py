"""Independent pins of the band-model reference's forward pass and its
quantised backward pass (oracle/mlp.py).

* Closed form: weights planted so that the network computes a sum that can be
  written out by hand.  Every planted weight is exact in bfloat16, and the
  first layer's pattern is not symmetric, so a transposed weight layout, a
  bias taken from the wrong offset or a lost ReLU changes the value.
* Autograd: the same network written with torch.nn.functional.linear in
  float64, the bfloat16 rounding taken as a straight-through step
  (W + (round(W) - W).detach(), rounded by torch's own bfloat16 conversion),
  and the pinball loss written as torch.where; torch's autograd gives the loss
  and the gradient that the hand-written backward pass must equal.  This
  checks the quantised backward (quantize=True), which finite differences
  cannot: the rounding makes the loss piecewise constant in the weights.
* Hand-derived gradients for weights that make most terms vanish, including a
  residual of exactly zero (the pinball subgradient takes the tau branch).
* Planted mistakes: each case rewrites one line of a copy of oracle/mlp.py and
  checks that these pins reject it.
"""
import importlib.util
import os
import sys

import numpy as np
import pytest
import torch

from oracle import mlp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mlp.py")

SIZES = [64 * 259, 64, 64 * 64, 64, 64, 1]


def _torch_net(flat: torch.Tensor, X: torch.Tensor, quantize: bool):
    """float64 network on the documented flat layout: W1[64][259] (row = hidden
    unit), b1, W2[64][64], b2, w3, b3."""
    W1, b1, W2, b2, w3, b3 = torch.split(flat, SIZES)
    W1 = W1.reshape(64, 259)
    W2 = W2.reshape(64, 64)

    def q(W):
        if not quantize:
            return W
        r = W.detach().to(torch.float32).to(torch.bfloat16).to(torch.float64)
        return W + (r - W).detach()  # value of the rounding, gradient of the identity

    h1 = torch.relu(torch.nn.functional.linear(X, q(W1), b1))
    h2 = torch.relu(torch.nn.functional.linear(h1, q(W2), b2))
    return torch.nn.functional.linear(h2, q(w3).reshape(1, 64), b3).reshape(-1)


def _torch_loss_grad(params, X, y, tau, quantize=True):
    flat = torch.tensor(np.asarray(params, np.float64), requires_grad=True)
    Xt = torch.tensor(np.asarray(X, np.float64))
    yt = torch.tensor(np.asarray(y, np.float64))
    yhat = _torch_net(flat, Xt, quantize)
    u = yt - yhat
    loss = torch.where(u < 0, (tau - 1.0) * u, tau * u).mean()
    loss.backward()
    return float(loss.detach()), flat.grad.numpy(), yhat.detach().numpy()


def _planted():
    """W1[h][h+3] = 1 (hidden unit h reads input h+3), b1 = 0;
    W2[k][(k+1) % 64] = 2, b2 = 0; w3[k] = k; b3 = 0.5.  Then
    y = 0.5 + sum_k 2 k relu(x[3 + (k+1) % 64])."""
    p = np.zeros(mlp.N_PARAMS, np.float32)
    o = 0
    for h in range(64):
        p[o + h * 259 + h + 3] = 1.0
    o += 64 * 259 + 64
    for k in range(64):
        p[o + k * 64 + (k + 1) % 64] = 2.0
    o += 64 * 64 + 64
    p[o:o + 64] = np.arange(64, dtype=np.float32)
    p[o + 64] = 0.5
    return p


def _rand_params(seed):
    """Weights with bits below bfloat16's precision (so quantisation matters)
    and non-zero biases (so every bias takes part)."""
    rng = np.random.default_rng(seed)
    p = mlp.init_params(seed).astype(np.float64)
    o = 64 * 259
    p[o:o + 64] = rng.normal(size=64) * 0.3
    o += 64 + 64 * 64
    p[o:o + 64] = rng.normal(size=64) * 0.3
    p[-1] = 1.7
    p = p.astype(np.float32)
    assert not np.array_equal(mlp.bf16_round(p), p)
    return p


def _check_closed_form(mod) -> bool:
    rng = np.random.default_rng(4)
    X = rng.normal(size=(9, 259))
    y, _ = mod.forward(_planted(), X, True)
    ref = 0.5 + sum(2.0 * k * np.maximum(X[:, 3 + (k + 1) % 64], 0.0) for k in range(64))
    return np.allclose(y, ref, rtol=0, atol=1e-9)


def _check_autograd(mod) -> bool:
    for seed, tau, B in [(11, 0.9, 12), (12, 0.5, 5), (13, 0.1, 1)]:
        rng = np.random.default_rng(seed)
        p = _rand_params(seed)
        X = rng.normal(size=(B, 259)) * 0.5
        y = rng.normal(size=B) + 1.0
        for quantize in (True, False):
            l_ref, g_ref, yh_ref = _torch_loss_grad(p, X, y, tau, quantize)
            yh, _ = mod.forward(p, X, quantize)
            loss, g = mod.backward(p, X, y, tau, quantize)
            if not np.allclose(yh, yh_ref, rtol=1e-12, atol=1e-12):
                return False
            if abs(loss - l_ref) > 1e-12 * max(1.0, abs(l_ref)):
                return False
            if not np.allclose(g, g_ref, rtol=1e-10, atol=1e-13):
                return False
    return True


def _check_hand_gradients(mod) -> bool:
    """All weights zero except b2 = 1 and w3 = c: then A2 = 1, yhat = 64 c + b3
    for every row, and
      dL/db3 = -(1/B) sum_r t_r,  dL/dw3[k] = -(1/B) sum_r t_r,
      dL/db2[k] = -(1/B) sum_r t_r c[k],  every other entry 0,
    with t_r = tau if y_r >= yhat_r else tau - 1.  Row 0's target equals yhat
    exactly, so its residual is zero and it takes the tau branch."""
    B, tau = 6, 0.8
    c = (np.arange(64) % 5 - 2).astype(np.float32) * 0.25  # exact in bfloat16
    p = np.zeros(mlp.N_PARAMS, np.float32)
    o = 64 * 259 + 64 + 64 * 64
    p[o:o + 64] = 1.0
    p[o + 64:o + 128] = c
    p[-1] = 0.75
    yhat = float(c.astype(np.float64).sum()) + 0.75
    y = np.array([yhat, yhat + 1, yhat - 2, yhat + 0.5, yhat - 0.25, yhat + 3])
    X = np.random.default_rng(5).normal(size=(B, 259))
    t = np.where(y >= yhat, tau, tau - 1.0)
    loss, g = mod.backward(p, X, y, tau, True)
    exp = np.zeros(mlp.N_PARAMS)
    exp[o:o + 64] = -(t.sum() / B) * c
    exp[o + 64:o + 128] = -t.sum() / B
    exp[-1] = -t.sum() / B
    u = y - yhat
    exp_loss = float(np.mean(np.where(u < 0, (tau - 1) * u, tau * u)))
    return np.allclose(g, exp, rtol=0, atol=1e-12) and abs(loss - exp_loss) < 1e-12


PINS = [_check_closed_form, _check_autograd, _check_hand_gradients]


def test_forward_closed_form():
    assert _check_closed_form(mlp)


def test_forward_and_quantised_backward_match_autograd():
    assert _check_autograd(mlp)


def test_hand_derived_gradients():
    assert _check_hand_gradients(mlp)


MUTANTS = {
    "w1_layout_transposed": ("W1 = p[o:o + H1 * D_IN].reshape(H1, D_IN)",
                             "W1 = p[o:o + H1 * D_IN].reshape(D_IN, H1).T"),
    "bias_order_swapped": ("b1 = p[o:o + H1]; o += H1\n    W2 = p[o:o + H2 * H1].reshape(H2, H1); o += H2 * H1",
                           "W2 = p[o:o + H2 * H1].reshape(H2, H1); o += H2 * H1\n    b1 = p[o:o + H1]; o += H1"),
    "rounded_biases": ("Z1 = X @ qW1.T + b1.astype(np.float64)",
                       "Z1 = X @ qW1.T + q(b1).astype(np.float64)"),
    "second_relu_dropped": ("A2 = np.maximum(Z2, 0.0)", "A2 = Z2"),
    "backward_unrounded_w3": ("dA2 = np.outer(dy, qw3)", "dA2 = np.outer(dy, unpack(params)[4])"),
    "backward_unrounded_w2": ("dA1 = dZ2 @ qW2", "dA1 = dZ2 @ unpack(params)[2]"),
    "first_mask_dropped": ("dZ1 = dA1 * (Z1 > 0)", "dZ1 = dA1"),
    "mask_from_wrong_layer": ("dZ2 = dA2 * (Z2 > 0)", "dZ2 = dA2 * (A2 > 1e-3)"),
    "zero_residual_branch": ("dy = -np.where(u < 0, tau - 1.0, tau) / B",
                             "dy = -np.where(u <= 0, tau - 1.0, tau) / B"),
    "mean_dropped": ("dy = -np.where(u < 0, tau - 1.0, tau) / B", "dy = -np.where(u < 0, tau - 1.0, tau)"),
    "db3_mean": ("db3 = np.array([dy.sum()])", "db3 = np.array([dy.mean()])"),
    "dw1_from_activations": ("dW1 = dZ1.T @ X", "dW1 = dZ1.T @ np.maximum(X, 0)"),
    "b2_grad_unmasked": ("db2 = dZ2.sum(0)", "db2 = dA2.sum(0)"),
}


def _load_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found once"
    path = tmp_path / f"mlp_{name}.py"
    # the copy imports nothing from the oracle package
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"mlp_mut_{name}", str(path))
    mod = importlib.util.module_from_spec(spec)
    sys.modules[spec.name] = mod
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    mod = _load_mutant(name, tmp_path)
    passed = []
    for pin in PINS:
        try:
            passed.append(bool(pin(mod)))
        except (ValueError, IndexError, AssertionError):
            passed.append(False)
    assert not all(passed), f"mutant {name} slipped through the pins"
