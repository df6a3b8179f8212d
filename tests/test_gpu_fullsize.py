"""Parity at the benchmark workloads' full sizes, in the launch configuration
bench.py times, every output against the oracle: the 4096-pair batch (every
score and path), the 512-sequence all-pairs matrix (all 130,816 entries,
plus symmetry and the diagonal) and the 8192-pair learned-band batch (every
score and every path byte, and identical to full DP on the device).  The
oracle runs on all host threads in chunks, with a progress line after
each."""
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


def _chunks(cost, parts):
    """Split indices 0..len(cost)-1 into about `parts` runs of equal total cost."""
    cum = np.cumsum(np.asarray(cost, np.float64))
    edges = np.searchsorted(cum, np.linspace(0, cum[-1], parts + 1)[1:-1])
    return np.split(np.arange(len(cost)), np.unique(edges + 1))


def test_allpairs_512():
    seqs = config_allpairs()
    pool, off, lens = pack_seqs(seqs)
    say("full all-pairs: 512 sequences on the GPU")
    M = gpu_allpairs(pool, off, lens, int(lens.max()), P)
    assert (M == M.T).all()
    assert (np.diag(M) == lens.astype(np.int64) * P[0]).all()
    iu, ju = np.triu_indices(len(seqs), 1)
    cost = lens[iu].astype(np.float64) * lens[ju]
    for c, sel in enumerate(_chunks(cost, 8)):
        s_ref, _ = oracle.align_batch(pool, off[iu[sel]], lens[iu[sel]], off[ju[sel]], lens[ju[sel]], P,
                                      with_paths=False)
        bad = np.nonzero(M[iu[sel], ju[sel]] != s_ref)[0]
        assert len(bad) == 0, [(int(iu[sel][k]), int(ju[sel][k])) for k in bad[:8]]
        say(f"full all-pairs: oracle chunk {c + 1}/8 equal ({len(sel)} entries)")


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
    # every pair against the oracle: score, path length and every path byte
    s_h, p_h, o_h, l_h = s.cpu().numpy(), p.cpu().numpy(), poff.cpu().numpy(), plen.cpu().numpy()
    pool, ao, al, bo, bl = pack_pairs(test)
    cost = al.astype(np.float64) * bl
    parts = _chunks(cost, 8)
    for c, sel in enumerate(parts):
        ref_s, ref_p = oracle.align_batch(pool, ao[sel], al[sel], bo[sel], bl[sel], P)
        for q, k in enumerate(sel):
            assert s_h[k] == ref_s[q], (k, s_h[k], ref_s[q])
            assert l_h[k] == len(ref_p[q]), k
            assert np.array_equal(p_h[o_h[k]:o_h[k] + l_h[k]], ref_p[q]), k
        say(f"learned band: oracle chunk {c + 1}/{len(parts)} equal ({len(sel)} pairs)")
