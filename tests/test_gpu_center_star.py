"""Centre-star multiple alignment on the GPU against the oracle (oracle/msa.py):
the centre, the width and every byte of the alignment, on small families;
at the all-pairs workload's full size (512 sequences of 500..5000 bases),
properties that hold at any size plus every row against the oracle's own
pairwise alignment to the centre."""
import numpy as np
import pytest

import oracle
from oracle import msa as omsa
from workloads import config_allpairs, mutate, pack_seqs, random_seq

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2412_21103_amd as nwp  # noqa: E402
from gpu_util import say  # noqa: E402

P = (1, -1, -1)
GAP = 255


def _dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")


def _gpu_center_star(seqs, scoring=P, width_cap=None):
    pool, off, lens = pack_seqs(seqs)
    ml = max(int(lens.max()) if len(lens) else 1, 1)
    dp, do, dl = _dev(pool if len(pool) else np.zeros(1, np.uint8), np.uint8), _dev(off, np.int64), _dev(lens, np.int32)
    S = nwp.allpairs(dp, do, dl, ml, scoring)
    c, M, w = nwp.center_star(dp, do, dl, ml, S, scoring, gap_byte=GAP, width_cap=width_cap)
    torch.cuda.synchronize()
    return S.cpu().numpy(), int(c.item()), M.cpu().numpy(), int(w.item())


def _family(seed, nseq, lo, hi, rate_hi=0.25):
    rng = np.random.default_rng(seed)
    root = random_seq(rng, hi + 300)
    return [mutate(rng, root, float(rng.uniform(0.02, rate_hi)))[: int(rng.integers(lo, hi + 1))].copy()
            for _ in range(nseq)]


@pytest.mark.parametrize("seed,nseq,lo,hi", [(11, 1, 30, 30), (12, 2, 1, 40), (13, 5, 0, 60), (14, 17, 50, 300),
                                             (15, 40, 200, 700), (16, 8, 600, 1600)])
def test_center_star_matches_oracle(seed, nseq, lo, hi):
    seqs = _family(seed, nseq, lo, hi)
    say(f"center star: {nseq} sequences of {lo}..{hi}")
    S, c, M, w = _gpu_center_star(seqs)
    pool, off, lens = pack_seqs(seqs)
    assert np.array_equal(S, oracle.allpairs(pool, off, lens, P))
    c_ref, M_ref = omsa.center_star(seqs, P, gap_byte=GAP, scores=S)
    assert c == c_ref
    assert w == M_ref.shape[1]
    assert np.array_equal(M[:, :w], M_ref)


def test_center_star_identical_and_other_scoring():
    rng = np.random.default_rng(21)
    s = random_seq(rng, 333)
    seqs = [s.copy() for _ in range(4)] + [mutate(rng, s, 0.2)]
    for sc in (P, (2, -3, -2)):
        S, c, M, w = _gpu_center_star(seqs, sc)
        c_ref, M_ref = omsa.center_star(seqs, sc, gap_byte=GAP, scores=S)
        assert c == c_ref and w == M_ref.shape[1] and np.array_equal(M[:, :w], M_ref), sc


def test_center_star_small_buffer_reports_width_only():
    seqs = _family(31, 6, 100, 200)
    _, _, M_full, w = _gpu_center_star(seqs)
    pool, off, lens = pack_seqs(seqs)
    dp, do, dl = _dev(pool, np.uint8), _dev(off, np.int64), _dev(lens, np.int32)
    ml = int(lens.max())
    S = nwp.allpairs(dp, do, dl, ml, P)
    c, M, w2 = nwp.center_star(dp, do, dl, ml, S, P, gap_byte=GAP, width_cap=w - 1)
    M.fill_(7)
    c, M2, w2 = nwp.center_star(dp, do, dl, ml, S, P, gap_byte=GAP, width_cap=w - 1)
    torch.cuda.synchronize()
    assert int(w2.item()) == w
    # the rows are left alone when the width exceeds the buffer
    _, M3, _ = nwp.center_star(dp, do, dl, ml, S, P, gap_byte=GAP, width_cap=w)
    torch.cuda.synchronize()
    assert np.array_equal(M3.cpu().numpy(), M_full[:, :w])


def _induced(row_c, row_k):
    both = (row_c != GAP) | (row_k != GAP)
    rc, rk = row_c[both], row_k[both]
    return np.where((rc != GAP) & (rk != GAP), oracle.D, np.where(rk == GAP, oracle.U, oracle.L)).astype(np.uint8)


def test_center_star_allpairs_full_size():
    seqs = config_allpairs()
    pool, off, lens = pack_seqs(seqs)
    say(f"center star at full size: {len(seqs)} sequences")
    S, c, M, w = _gpu_center_star(seqs)
    assert c == omsa.center_index(S)
    lc = len(seqs[c])
    ins = np.zeros(lc + 1, np.int64)
    for k in range(len(seqs)):
        row = M[k, :w]
        assert row[row != GAP].tolist() == seqs[k].tolist(), k
        if k == c:
            continue
        path = _induced(M[c, :w], row)
        r, ok = oracle.rescore(path, seqs[c], seqs[k], P)
        assert ok and r == S[c, k], k
        # insertion runs per slot
        slot, cnt = 0, np.zeros(lc + 1, np.int64)
        for mv in path.tolist():
            if mv == oracle.L:
                cnt[slot] += 1
            else:
                slot += 1
        ins = np.maximum(ins, cnt)
    assert w == lc + int(ins.sum())
    # every row against the oracle's own alignment of that sequence to the
    # centre (511 pairwise alignments on all host threads)
    others = [k for k in range(len(seqs)) if k != c]
    say(f"center star: oracle pairwise paths for all {len(others)} rows")
    a_pool = np.concatenate([seqs[c]] + [seqs[k] for k in others]).astype(np.uint8)
    lens_o = np.array([len(seqs[k]) for k in others], np.int32)
    b_off = len(seqs[c]) + np.concatenate([[0], np.cumsum(lens_o)[:-1]]).astype(np.int64)
    s_ref, p_ref = oracle.align_batch(a_pool, np.zeros(len(others), np.int64), np.full(len(others), lc, np.int32),
                                      b_off, lens_o, P)
    for q, k in enumerate(others):
        assert s_ref[q] == S[c, k], k
        assert _induced(M[c, :w], M[k, :w]).tolist() == p_ref[q].tolist(), k
