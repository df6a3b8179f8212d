"""Scoring constants beyond a signed byte.  The one-hot lookup holds each
cell's diagonal terms, 4(s - 2 gap) + 2 with directions and s - 2 gap
without, as signed bytes; a call whose terms do not fit runs every pair
through the byte-comparing sweep, which holds them in 23 bits.  Every entry
point must still agree with the oracle, on nucleotide codes (which would
otherwise take the one-hot lookup)."""
import numpy as np
import pytest

import oracle
from oracle import coopt
from workloads import Pairs, pack_pairs, pack_seqs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2412_21103_amd as nwp  # noqa: E402
from gpu_util import gpu_align, gpu_allpairs, gpu_batch, say  # noqa: E402

# (50, -40, -30): terms 442 / 82 with directions, 110 / 20 without;
# (5, -200, -3): terms 46 / -774 with directions, 11 / -194 without.
SCORINGS = [(50, -40, -30), (5, -200, -3)]


def _dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")


def _pairs(seed, npairs, lo, hi):
    rng = np.random.default_rng(seed)
    A, B = [], []
    for _ in range(npairs):
        a = rng.integers(0, 4, int(rng.integers(lo, hi))).astype(np.uint8)
        b = a.copy()
        k = rng.random(len(b)) < 0.15
        b[k] = rng.integers(0, 4, int(k.sum())).astype(np.uint8)
        cut = int(rng.integers(0, max(len(b) // 8, 1)))
        b = np.concatenate([b[cut:], rng.integers(0, 4, int(rng.integers(0, 30))).astype(np.uint8)])
        A.append(a)
        B.append(b)
    return Pairs(A, B, "wide-scoring")


@pytest.mark.parametrize("sc", SCORINGS)
def test_single_pairs_wide_scoring(sc):
    rng = np.random.default_rng(1)
    for m, n in [(300, 280), (700, 650), (1, 900), (0, 5)]:
        say(f"wide scoring {sc}: single {m}x{n}")
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = rng.integers(0, 4, n).astype(np.uint8)
        s_ref, p_ref = oracle.align(a, b, sc)
        s, p = gpu_align(a, b, sc)
        assert s == s_ref and p.tolist() == p_ref.tolist(), (m, n)
        s2, _ = gpu_align(a, b, sc, score_only=True)
        assert s2 == s_ref, (m, n)


@pytest.mark.parametrize("sc", SCORINGS)
def test_batch_and_band_wide_scoring(sc):
    pairs = _pairs(2, 40, 50, 900)
    pool, ao, al, bo, bl = pack_pairs(pairs)
    ml = int(max(al.max(), bl.max()))
    s_ref, p_ref = oracle.align_batch(pool, ao, al, bo, bl, sc)
    say(f"wide scoring {sc}: batch")
    s, paths, plen = gpu_batch(pool, ao, al, bo, bl, ml, sc)
    assert np.array_equal(s, s_ref)
    for k in range(len(pairs)):
        assert paths[k].tolist() == p_ref[k].tolist(), k
    for w0, doubling in [(0, False), (8, True)]:
        say(f"wide scoring {sc}: banded from {w0}, doubling {doubling}")
        out = nwp.align_batch_banded(_dev(pool, np.uint8), _dev(ao, np.int64), _dev(al, np.int32),
                                     _dev(bo, np.int64), _dev(bl, np.int32), ml, sc, w_default=w0,
                                     doubling=doubling)
        torch.cuda.synchronize()
        s, pth, poff, pl = (t.cpu().numpy() for t in out[:4])
        assert np.array_equal(s, s_ref)
        for k in range(len(pairs)):
            assert pth[poff[k]:poff[k] + pl[k]].tolist() == p_ref[k].tolist(), (w0, k)


@pytest.mark.parametrize("sc", SCORINGS)
def test_allpairs_and_cooptimal_wide_scoring(sc):
    rng = np.random.default_rng(3)
    seqs = [rng.integers(0, 4, int(rng.integers(0, 500))).astype(np.uint8) for _ in range(14)]
    pool, off, lens = pack_seqs(seqs)
    say(f"wide scoring {sc}: all-pairs")
    M = gpu_allpairs(pool, off, lens, max(1, int(lens.max())), sc)
    assert np.array_equal(M, oracle.allpairs(pool, off, lens, sc))
    pairs = _pairs(4, 24, 20, 160)
    pool, ao, al, bo, bl = pack_pairs(pairs)
    ml = max(1, int(max(al.max(), bl.max())))
    say(f"wide scoring {sc}: co-optimal counts")
    d = [_dev(pool, np.uint8), _dev(ao, np.int64), _dev(al, np.int32), _dev(bo, np.int64), _dev(bl, np.int32)]
    out = nwp.cooptimal(*d, ml, sc, k=2)
    torch.cuda.synchronize()
    scores, counts, sat = (o.cpu().numpy() for o in out[:3])
    s_ref, c_ref, f_ref = coopt.count_batch(pool, ao, al, bo, bl, sc)
    assert np.array_equal(scores, s_ref)
    assert np.array_equal(counts.view(np.uint64), c_ref)
    assert np.array_equal(sat, f_ref)


@pytest.mark.parametrize("sc", SCORINGS)
def test_center_star_wide_scoring(sc):
    from oracle import msa as omsa
    rng = np.random.default_rng(7)
    root = rng.integers(0, 4, 500).astype(np.uint8)
    seqs = []
    for _ in range(10):
        s = root.copy()
        k = rng.random(len(s)) < 0.1
        s[k] = rng.integers(0, 4, int(k.sum())).astype(np.uint8)
        keep = rng.random(len(s)) >= 0.03
        seqs.append(s[keep][: int(rng.integers(200, 500))].copy())
    pool, off, lens = pack_seqs(seqs)
    ml = int(lens.max())
    say(f"wide scoring {sc}: centre star")
    dp, do, dl = _dev(pool, np.uint8), _dev(off, np.int64), _dev(lens, np.int32)
    S = nwp.allpairs(dp, do, dl, ml, sc)
    c, M, w = nwp.center_star(dp, do, dl, ml, S, sc, gap_byte=255)
    torch.cuda.synchronize()
    c_ref, M_ref = omsa.center_star(seqs, sc, gap_byte=255, scores=S.cpu().numpy())
    assert np.array_equal(S.cpu().numpy(), oracle.allpairs(pool, off, lens, sc))
    assert int(c.item()) == c_ref
    w = int(w.item())
    assert w == M_ref.shape[1]
    assert np.array_equal(M.cpu().numpy()[:, :w], M_ref)
