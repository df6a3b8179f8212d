"""Parity at the benchmark workloads' full sizes, in the launch configuration
bench.py times: the 4096-pair batch (every pair against the oracle), the
512-sequence all-pairs matrix (symmetry, diagonal, a 48-sequence block and
random entries against the oracle) and the 8192-pair learned-band batch
(identical to full DP on the device, a sample against the oracle)."""
import numpy as np
import pytest

import oracle
from workloads import config_allpairs, config_band_batch, config_batch, pack_pairs, pack_seqs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2412_21103_amd as nwp  # noqa: E402
from paper_2412_21103_amd import band_model  # noqa: E402
from gpu_util import gpu_allpairs, gpu_batch, say  # noqa: E402

P = oracle.PAPER_SCORING


def _dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")


def test_batch_4096_every_pair():
    pairs = config_batch()
    pool, ao, al, bo, bl = pack_pairs(pairs)
    ml = int(max(al.max(), bl.max()))
    say(f"full batch: {len(pairs)} pairs on the GPU")
    s, paths, plen = gpu_batch(pool, ao, al, bo, bl, ml, P)
    say("full batch: oracle on every pair")
    s_ref, p_ref = oracle.align_batch(pool, ao, al, bo, bl, P)
    assert (s == s_ref).all(), np.nonzero(s != s_ref)[0][:8]
    bad = [k for k in range(len(pairs)) if paths[k].tolist() != p_ref[k].tolist()]
    assert not bad, bad[:8]
    s2, _ = gpu_batch(pool, ao, al, bo, bl, ml, P, score_only=True)
    assert (s2 == s_ref).all()


def test_allpairs_512():
    seqs = config_allpairs()
    pool, off, lens = pack_seqs(seqs)
    say("full all-pairs: 512 sequences on the GPU")
    M = gpu_allpairs(pool, off, lens, int(lens.max()), P)
    assert (M == M.T).all()
    assert (np.diag(M) == lens.astype(np.int64) * P[0]).all()
    say("full all-pairs: oracle on the first 48 sequences")
    sub = seqs[:48]
    sp, so, sl = pack_seqs(sub)
    assert (M[:48, :48] == oracle.allpairs(sp, so, sl, P)).all()
    rng = np.random.default_rng(1)
    say("full all-pairs: oracle on 40 random entries")
    for _ in range(40):
        i, j = (int(x) for x in rng.integers(0, len(seqs), 2))
        assert M[i, j] == oracle.score(seqs[i], seqs[j], P), (i, j)


def test_learned_band_8192():
    say("learned band: generating 8192 + 2048 pairs")
    test = config_band_batch()
    train = config_band_batch(seed=5100, npairs=2048)
    d = [_dev(x, dt) for x, dt in zip(pack_pairs(test), (np.uint8, np.int64, np.int32, np.int64, np.int32))]
    ml = int(max(d[2].max().item(), d[4].max().item()))
    dt = [_dev(x, t) for x, t in zip(pack_pairs(train), (np.uint8, np.int64, np.int32, np.int64, np.int32))]
    mlt = int(max(dt[2].max().item(), dt[4].max().item()))
    x, _, _, target = band_model.features_and_labels(*dt, mlt)
    mlp, _ = band_model.train(x, target, epochs=100, batch=256, lr=3e-3, tau=0.9, seed=1)
    del dt, x, target
    ws = torch.empty(nwp.learned_workspace_size(len(test), ml), dtype=torch.uint8, device="cuda")
    say("learned band: full DP and learned band on the GPU")
    s_ref, p_ref, poff, plen_ref = nwp.align_batch(*d, ml, workspace=ws)
    s, p, _, plen, _, status, cells = nwp.align_batch_learned(*d, ml, mlp, 0.1, path_off=poff, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(s, s_ref) and torch.equal(plen, plen_ref)
    plen64 = plen_ref.to(torch.int64)
    starts = torch.repeat_interleave(poff, plen64)
    base = torch.repeat_interleave(torch.cumsum(plen64, 0) - plen64, plen64)
    idx = starts + torch.arange(int(plen64.sum()), device="cuda") - base
    assert torch.equal(p[idx], p_ref[idx])
    full_cells = float((d[2].double() * d[4].double()).sum())
    assert float(cells.sum()) < 0.6 * full_cells
    # a sample against the oracle: four random pairs and the two largest
    s_h, p_h, o_h, l_h = s.cpu().numpy(), p.cpu().numpy(), poff.cpu().numpy(), plen.cpu().numpy()
    rng = np.random.default_rng(2)
    cost = np.array([len(a) * len(b) for a, b in zip(test.a, test.b)])
    sample = list(rng.choice(len(test), 4, replace=False)) + list(np.argsort(cost)[-2:])
    say(f"learned band: oracle on pairs {sample}")
    pool, ao, al, bo, bl = pack_pairs(test)
    sel = np.array(sample)
    ref_s, ref_p = oracle.align_batch(pool, ao[sel], al[sel], bo[sel], bl[sel], P)
    for q, k in enumerate(sample):
        assert s_h[k] == ref_s[q], k
        assert p_h[o_h[k]:o_h[k] + l_h[k]].tolist() == ref_p[q].tolist(), k
