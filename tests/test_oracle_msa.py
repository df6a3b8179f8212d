"""Pins for the center-star oracle (oracle/msa.py), independent of its code:

* the center is the brute-force argmax of off-diagonal row sums, lowest index
  on ties;
* every row, gaps removed, is its input sequence;
* the alignment induced between the center row and row k (columns where both
  are gaps dropped) is exactly the oracle's pairwise path;
* the result equals a direct construction: each insertion slot of the center
  is as wide as the largest insertion any sequence makes there, every row's
  inserted residues sit left-justified in the slot, and the width is
  len(center) + the sum of the slot widths;
* merging in another order gives the same alignment.
"""
import numpy as np
import pytest

import oracle
from oracle import msa
from workloads import mutate, random_seq

GAP = 255


def _family(seed, nseq, lo, hi, rate_hi=0.25):
    rng = np.random.default_rng(seed)
    root = random_seq(rng, hi + 200)
    out = []
    for _ in range(nseq):
        d = mutate(rng, root, float(rng.uniform(0.02, rate_hi)))
        out.append(d[: int(rng.integers(lo, hi + 1))].copy())
    return out


def _brute_center(S):
    n = len(S)
    best, arg = None, 0
    for i in range(n):
        t = sum(int(S[i][j]) for j in range(n) if j != i)
        if best is None or t > best:
            best, arg = t, i
    return arg


def _direct(seqs, c, paths):
    """Slot widths = max insertion length; rows left-justified in slots."""
    lc = len(seqs[c])
    ins = np.zeros(lc + 1, np.int64)
    per = {}
    for k, path in paths.items():
        slot, run, cnt = 0, 0, np.zeros(lc + 1, np.int64)
        for mv in path.tolist():
            if mv == oracle.L:
                cnt[slot] += 1
            else:
                slot += 1
        per[k] = cnt
        ins = np.maximum(ins, cnt)
    start = np.zeros(lc + 1, np.int64)   # first column of slot p
    col = np.zeros(lc, np.int64)          # column of center residue p
    x = 0
    for p in range(lc + 1):
        start[p] = x
        x += ins[p]
        if p < lc:
            col[p] = x
            x += 1
    width = x
    out = np.full((len(seqs), width), GAP, np.uint8)
    out[c, col] = seqs[c]
    for k, path in paths.items():
        p, t, j = 0, 0, 0
        for mv in path.tolist():
            if mv == oracle.L:
                out[k, start[p] + t] = seqs[k][j]
                t += 1
                j += 1
            else:
                if mv == oracle.D:
                    out[k, col[p]] = seqs[k][j]
                    j += 1
                p += 1
                t = 0
    return out


def _induced(row_c, row_k):
    mv = []
    for x, y in zip(row_c.tolist(), row_k.tolist()):
        if x == GAP and y == GAP:
            continue
        mv.append(oracle.D if (x != GAP and y != GAP) else (oracle.U if y == GAP else oracle.L))
    return mv


@pytest.mark.parametrize("seed,nseq,lo,hi", [(1, 2, 5, 12), (2, 6, 1, 30), (3, 12, 20, 80), (4, 9, 0, 15)])
def test_center_star_pins(seed, nseq, lo, hi):
    seqs = _family(seed, nseq, lo, hi)
    lens = np.array([len(s) for s in seqs], np.int32)
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    pool = np.concatenate(seqs) if sum(lens) else np.zeros(0, np.uint8)
    S = oracle.allpairs(pool, off, lens)
    c, M = msa.center_star(seqs, gap_byte=GAP, scores=S)
    assert c == _brute_center(S)
    assert M.shape[0] == nseq
    for k in range(nseq):
        row = M[k]
        assert row[row != GAP].tolist() == seqs[k].tolist(), k
    paths = msa.pairwise_to_center(seqs, c)
    for k, path in paths.items():
        assert _induced(M[c], M[k]) == path.tolist(), k
    assert np.array_equal(M, _direct(seqs, c, paths))
    # another merge order: the alignment does not depend on it
    M2 = msa.merge(seqs, c, paths, GAP, order=sorted(paths, reverse=True))
    assert np.array_equal(M, M2)


def test_center_star_single_and_identical():
    rng = np.random.default_rng(9)
    s = random_seq(rng, 17)
    c, M = msa.center_star([s], gap_byte=GAP)
    assert c == 0 and M.tolist() == [s.tolist()]
    c, M = msa.center_star([s, s.copy(), s.copy()], gap_byte=GAP)
    assert c == 0 and all(M[k].tolist() == s.tolist() for k in range(3))


def test_center_tie_goes_to_lowest_index():
    S = np.array([[0, 5, 5], [5, 0, 5], [5, 5, 0]], np.int32)
    assert msa.center_index(S) == 0
    S = np.array([[9, 1, 2], [1, 9, 4], [2, 4, 9]], np.int32)
    assert msa.center_index(S) == 2
