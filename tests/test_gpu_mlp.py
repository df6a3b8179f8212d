"""Band-model kernels against the float64 reference in oracle/mlp.py and
oracle/band.py: features, forward, half-widths, labels, gradients and Adam.

Tolerances: features are exact up to float32 division (rtol 1e-6); the
forward pass agrees within abs 1e-4 + rel 1e-4 (float32 sums in another
order); gradients within 1e-3 of the gradient's norm, and per element within
rel 1e-3 plus 2e-5 of the entry's sum of absolute terms (float32 summation
order); Adam
within a few float32 ulps; the bfloat16 copy and every integer output
exactly."""
import numpy as np
import pytest

import oracle
from oracle import band, mlp as omlp
from workloads import config_band_batch, mutate, pack_pairs, random_seq, Pairs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2412_21103_amd as nwp  # noqa: E402
from gpu_util import say  # noqa: E402

P = (1, -1, -1)


def _dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")


def _pairs_dev(pairs):
    pool, ao, al, bo, bl = pack_pairs(pairs)
    return (_dev(pool, np.uint8), _dev(ao, np.int64), _dev(al, np.int32), _dev(bo, np.int64),
            _dev(bl, np.int32), int(max(al.max(), bl.max(), 1)))


def _edge_pairs():
    rng = np.random.default_rng(91)
    A, B = [], []
    for m, n in [(0, 0), (0, 5), (3, 3), (4, 3), (4, 4), (5, 9), (7, 0), (1023, 1024), (1025, 1029),
                 (2047, 2100), (3001, 2990)]:
        a = random_seq(rng, m)
        b = mutate(rng, a, 0.1)[:n] if n <= m else np.concatenate([a, random_seq(rng, n - m)])
        if len(b) < n:
            b = np.concatenate([b, random_seq(rng, n - len(b))])
        A.append(a)
        B.append(b)
    more = config_band_batch(seed=92, npairs=24, lo=200, hi=4000)
    return Pairs(A + more.a, B + more.b, "mlp_edges")


@pytest.fixture(scope="module")
def pairs():
    return _edge_pairs()


@pytest.fixture(scope="module")
def params():
    p = omlp.init_params(7)
    rng = np.random.default_rng(8)
    # non-zero biases so every term of the forward pass is exercised
    W1, b1, W2, b2, w3, b3 = omlp.unpack(p)
    b1[:] = rng.uniform(-0.2, 0.2, b1.shape)
    b2[:] = rng.uniform(-0.2, 0.2, b2.shape)
    b3[:] = 0.5
    return p


def test_features_match_reference(pairs):
    say("mlp: features")
    d = _pairs_dev(pairs)
    x = nwp.mlp_features(*d[:5]).cpu().numpy()
    ref = np.stack([omlp.features(a, b) for a, b in zip(pairs.a, pairs.b)])
    assert x.shape == ref.shape
    np.testing.assert_allclose(x, ref, rtol=1e-6, atol=0)
    # the count differences themselves are integers
    den = np.maximum(np.maximum([len(a) for a in pairs.a], [len(b) for b in pairs.b]), 1)
    cnt = x[:, 3:].astype(np.float64) * den[:, None]
    assert np.abs(cnt - np.rint(cnt)).max() < 1e-3


def test_bf16_copy_bits(params):
    say("mlp: bfloat16 copy")
    m = nwp.Mlp(params)
    torch.cuda.synchronize()
    got = m.params_bf16.cpu().numpy().view(np.uint16)
    want = (omlp.bf16_round(params).view(np.uint32) >> 16).astype(np.uint16)
    assert (got == want).all()


def test_forward_matches_reference(pairs, params):
    say("mlp: forward")
    d = _pairs_dev(pairs)
    x = nwp.mlp_features(*d[:5])
    m = nwp.Mlp(params)
    y = nwp.mlp_forward(m, x).cpu().numpy()
    ref, _ = omlp.forward(params, x.cpu().numpy().astype(np.float64))
    np.testing.assert_allclose(y, ref, rtol=1e-4, atol=1e-4)
    # many rows (grid-strided waves) and random inputs with wider spread
    rng = np.random.default_rng(5)
    X = rng.normal(0, 0.3, size=(3001, omlp.D_IN)).astype(np.float32)
    y2 = nwp.mlp_forward(m, _dev(X, np.float32)).cpu().numpy()
    ref2, _ = omlp.forward(params, X.astype(np.float64))
    np.testing.assert_allclose(y2, ref2, rtol=1e-4, atol=1e-4)


def test_widths_match_reference():
    say("mlp: widths")
    rng = np.random.default_rng(6)
    n = 4000
    yhat = np.concatenate([rng.uniform(-3, 12, n - 6), [0.0, -0.0, 1e-8, 30.0, np.log1p(7.0), 88.0]])
    yhat = yhat.astype(np.float32)
    al = rng.integers(0, 20001, yhat.size).astype(np.int32)
    bl = rng.integers(0, 20001, yhat.size).astype(np.int32)
    for margin in [np.float32(0.0), np.float32(0.1), np.float32(0.37)]:
        w = nwp.mlp_widths(_dev(yhat, np.float32), _dev(al, np.int32), _dev(bl, np.int32),
                           float(margin)).cpu().numpy()
        ref = omlp.predict_width(yhat.astype(np.float64), al.astype(np.int64), bl.astype(np.int64),
                                 float(margin))
        assert (w == ref).all(), np.nonzero(w != ref)[0][:8]


def test_labels_match_reference(pairs):
    say("mlp: band labels")
    d = _pairs_dev(pairs)
    for sc in [P, (2, -3, -2), (3, 1, -1)]:
        s, _, _, _ = nwp.align_batch(*d, sc, score_only=True)
        w, t = nwp.band_labels(s, d[2], d[4], sc)
        s, w, t = s.cpu().numpy(), w.cpu().numpy(), t.cpu().numpy()
        for k, (a, b) in enumerate(zip(pairs.a, pairs.b)):
            assert s[k] == oracle.score(a, b, sc)
            assert w[k] == band.w_cert(int(s[k]), len(a), len(b), sc), (sc, k)
        np.testing.assert_allclose(t, np.log1p(w.astype(np.float64)), rtol=1e-6, atol=0)


def test_path_labels_match_oracle(pairs):
    # w_path of the oracle's own paths, against the device labels of the
    # device paths (the paths are identical, checked here too); two scorings
    # and an empty pair
    say("mlp: path labels")
    from workloads import Pairs
    ext = Pairs(list(pairs.a) + [np.zeros(0, np.uint8), pairs.a[0][:5]],
                list(pairs.b) + [pairs.b[1][:9], np.zeros(0, np.uint8)], "labels")
    d = _pairs_dev(ext)
    for sc in [P, (2, -3, -2)]:
        s, paths, poff, plen = nwp.align_batch(*d, sc)
        w, t = nwp.path_labels(paths, poff, plen, d[2], d[4])
        w, t = w.cpu().numpy(), t.cpu().numpy()
        for k, (a, b) in enumerate(zip(ext.a, ext.b)):
            s_ref, p_ref = oracle.align(a, b, sc)
            assert w[k] == band.w_path(p_ref, len(a), len(b)), (sc, k)
        np.testing.assert_allclose(t, np.log1p(w.astype(np.float64)), rtol=1e-6, atol=0)
    assert w.max() > 0


def _train_data(pairs, seed=11):
    d = _pairs_dev(pairs)
    x = nwp.mlp_features(*d[:5])
    rng = np.random.default_rng(seed)
    target = rng.uniform(0, 6, x.shape[0]).astype(np.float32)
    return x, _dev(target, np.float32)


def _abs_terms(params, X, tau):
    """Per gradient entry, the sum of the absolute values of the terms the
    backward pass adds up (the same chain with every factor made absolute):
    the scale of its float32 rounding error."""
    _, (X, Z1, A1, Z2, A2, qW2, qw3) = omlp.forward(params, X, True)
    B = X.shape[0]
    dy = np.full(B, max(tau, 1.0 - tau) / B)
    dA2 = np.outer(dy, np.abs(qw3))
    dZ2 = dA2 * (Z2 > 0)
    dA1 = dZ2 @ np.abs(qW2)
    dZ1 = dA1 * (Z1 > 0)
    return np.concatenate([(dZ1.T @ np.abs(X)).ravel(), dZ1.sum(0), (dZ2.T @ A1).ravel(), dZ2.sum(0),
                           A2.T @ dy, [dy.sum()]])


def test_gradient_matches_reference(pairs, params):
    say("mlp: gradient")
    x, target = _train_data(pairs)
    X = x.cpu().numpy().astype(np.float64)
    T = target.cpu().numpy().astype(np.float64)
    m = nwp.Mlp(params)
    for tau in [0.9, 0.5]:
        loss, grad = nwp.mlp_train_step(m, x, target, tau, 0.0, want_grad=True)
        loss_ref, grad_ref = omlp.backward(params, X, T, tau)
        g = grad.cpu().numpy().astype(np.float64)
        assert abs(float(loss.item()) - loss_ref) <= 1e-5 * max(1.0, abs(loss_ref))
        assert np.linalg.norm(g - grad_ref) <= 1e-3 * np.linalg.norm(grad_ref)
        # per element: rel 1e-3, plus a floor for float32 summation order that
        # scales with the sum of the absolute terms of that entry
        tol = 1e-3 * np.abs(grad_ref) + 2e-5 * _abs_terms(params, X, tau)
        bad = np.nonzero(np.abs(g - grad_ref) > tol)[0]
        assert bad.size == 0, (tau, bad[:8], g[bad[:8]], grad_ref[bad[:8]])
    assert m.step == 0  # lr == 0: no update
    # a gathered minibatch equals the reference on those rows
    rows = np.array([5, 0, 17, 17, 30, 2, 33], np.int32)
    loss, grad = nwp.mlp_train_step(m, x, target, 0.9, 0.0, rows=_dev(rows, np.int32), want_grad=True)
    loss_ref, grad_ref = omlp.backward(params, X[rows], T[rows], 0.9)
    g = grad.cpu().numpy().astype(np.float64)
    assert abs(float(loss.item()) - loss_ref) <= 1e-5 * max(1.0, abs(loss_ref))
    assert np.linalg.norm(g - grad_ref) <= 1e-3 * np.linalg.norm(grad_ref)


def test_adam_matches_reference(pairs, params):
    say("mlp: adam")
    x, target = _train_data(pairs)
    m = nwp.Mlp(params)
    p = params.copy()
    mo = np.zeros_like(p)
    ve = np.zeros_like(p)
    lr = 1e-3
    for step in (1, 2, 3):
        # the gradient the step uses is the one at the current weights
        _, grad = nwp.mlp_train_step(m, x, target, 0.9, 0.0, want_grad=True)
        g = grad.cpu().numpy()
        _, grad2 = nwp.mlp_train_step(m, x, target, 0.9, lr, want_grad=True)
        assert (grad2.cpu().numpy() == g).all()  # deterministic gradient
        p, mo, ve = omlp.adam_step(p, mo, ve, g, step, lr)
        got = m.params.cpu().numpy()
        np.testing.assert_allclose(got, p, rtol=2e-6, atol=1e-9)
        np.testing.assert_allclose(m.adam_m.cpu().numpy(), mo, rtol=1e-5, atol=1e-12)
        np.testing.assert_allclose(m.adam_v.cpu().numpy(), ve, rtol=1e-5, atol=1e-18)
        bits = m.params_bf16.cpu().numpy().view(np.uint16)
        assert (bits == (omlp.bf16_round(got).view(np.uint32) >> 16).astype(np.uint16)).all()
        assert m.step == step
        # continue from the device state so rounding differences do not accumulate
        p = got
        mo = m.adam_m.cpu().numpy()
        ve = m.adam_v.cpu().numpy()


def test_epoch_equals_steps(pairs, params):
    say("mlp: epoch vs steps")
    x, target = _train_data(pairs)
    n = int(x.shape[0])
    order = np.random.default_rng(3).permutation(n).astype(np.int32)
    a = nwp.Mlp(params)
    losses = nwp.mlp_train_epoch(a, x, target, _dev(order, np.int32), 8, 0.9, 1e-3).cpu().numpy()
    b = nwp.Mlp(params)
    ref = []
    for i0 in range(0, n, 8):
        rows = _dev(order[i0:i0 + 8], np.int32)
        loss, _ = nwp.mlp_train_step(b, x, target, 0.9, 1e-3, rows=rows)
        ref.append(float(loss.item()))
    assert a.step == b.step == (n + 7) // 8
    assert (a.params.cpu().numpy() == b.params.cpu().numpy()).all()
    np.testing.assert_array_equal(losses, np.array(ref, np.float32))


def test_learned_band_is_exact(pairs, params):
    say("mlp: learned band parity")
    d = _pairs_dev(pairs)
    m = nwp.Mlp(params)
    for margin in [0.0, 0.5]:
        s, paths, poff, plen, wu, st, cells = nwp.align_batch_learned(*d, m, margin)
        s, paths, poff, plen = (t.cpu().numpy() for t in (s, paths, poff, plen))
        for k, (a, b) in enumerate(zip(pairs.a, pairs.b)):
            s_ref, p_ref = oracle.align(a, b, P)
            assert s[k] == s_ref, (margin, k)
            assert paths[poff[k]:poff[k] + plen[k]].tolist() == p_ref.tolist(), (margin, k)
