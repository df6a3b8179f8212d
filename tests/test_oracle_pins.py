"""Pins for the CPU oracle: brute force, closed forms, a textbook edit distance,
hand-worked grids and invariants.  None of these reuse the oracle's code."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import band
from pins import (all_paths, brute_force, max_score_leaving_band, path_score,
                  score_from_edit_distance)

HERE = os.path.dirname(os.path.abspath(__file__))
P = (1, -1, -1)
OTHER_SCORINGS = [(2, -3, -2), (1, 0, -1), (3, -1, -2), (5, -4, -3)]
CODE = {"A": 0, "C": 1, "G": 2, "T": 3}


def enc(s):
    return np.array([CODE[c] for c in s], dtype=np.uint8)


def test_delannoy_counts():
    # number of alignments of lengths (m, n) is the Delannoy number D(m, n)
    assert len(all_paths(6, 6)) == 8989
    assert len(all_paths(3, 3)) == 63
    assert len(all_paths(0, 5)) == 1


def test_hand_examples():
    data = json.load(open(os.path.join(HERE, "golden", "hand_examples.json")))
    for case in data["cases"]:
        a, b, sc = enc(case["a"]), enc(case["b"]), tuple(case["scoring"])
        H = oracle.fill(a, b, sc)
        assert H.tolist() == case["H"], case
        s, path = oracle.align(a, b, sc)
        assert s == case["score"]
        assert path.tolist() == case["path"]


@pytest.mark.parametrize("alphabet", [2, 4])
def test_brute_force_all_small_lengths(alphabet):
    rng = np.random.default_rng(11 + alphabet)
    for m in range(0, 7):
        for n in range(0, 7):
            reps = 3 if m * n >= 25 else 6
            for _ in range(reps):
                a = rng.integers(0, alphabet, m).astype(np.uint8)
                b = rng.integers(0, alphabet, n).astype(np.uint8)
                for sc in [P, (2, -3, -2)]:
                    s_bf, p_bf = brute_force(a, b, sc)
                    s, p = oracle.align(a, b, sc)
                    assert s == s_bf, (a, b, sc)
                    assert p.tolist() == p_bf.tolist(), (a, b, sc)
                    assert oracle.score(a, b, sc) == s_bf


def test_brute_force_exhaustive_binary():
    # every binary pair up to length 3 x 3
    import itertools
    for m in range(0, 4):
        for n in range(0, 4):
            for a in itertools.product([0, 1], repeat=m):
                for b in itertools.product([0, 1], repeat=n):
                    a_ = np.array(a, np.uint8)
                    b_ = np.array(b, np.uint8)
                    s_bf, p_bf = brute_force(a_, b_, P)
                    s, p = oracle.align(a_, b_, P)
                    assert (s, p.tolist()) == (s_bf, p_bf.tolist())


def test_identical_closed_form():
    rng = np.random.default_rng(1)
    for L in [0, 1, 2, 17, 300]:
        a = rng.integers(0, 4, L).astype(np.uint8)
        for sc in [P, (2, -3, -2)]:
            s, p = oracle.align(a, a.copy(), sc)
            assert s == L * sc[0]
            assert p.tolist() == [1] * L


def test_empty_sides():
    rng = np.random.default_rng(2)
    for n in [0, 1, 5, 40]:
        b = rng.integers(0, 4, n).astype(np.uint8)
        e = np.zeros(0, np.uint8)
        for sc in [P] + OTHER_SCORINGS:
            s, p = oracle.align(e, b, sc)
            assert s == n * sc[2] and p.tolist() == [3] * n
            s, p = oracle.align(b, e, sc)
            assert s == n * sc[2] and p.tolist() == [2] * n


def test_single_row_closed_form():
    # m = 1 with the paper's constants: 2 - n if a1 occurs in b (paired with its
    # rightmost occurrence), else -n with a1 against b_n.
    rng = np.random.default_rng(3)
    for n in range(1, 30):
        for _ in range(5):
            a = rng.integers(0, 4, 1).astype(np.uint8)
            b = rng.integers(0, 4, n).astype(np.uint8)
            s, p = oracle.align(a, b, P)
            occ = np.nonzero(b == a[0])[0]
            if occ.size:
                assert s == 2 - n
                k = int(occ[-1])
            else:
                assert s == -n
                k = n - 1
            expect = [3] * k + [1] + [3] * (n - 1 - k)
            assert p.tolist() == expect


@pytest.mark.parametrize("sc", [P] + OTHER_SCORINGS)
def test_weighted_edit_distance_identity(sc):
    rng = np.random.default_rng(4)
    for _ in range(25):
        m, n = rng.integers(0, 120, 2)
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = rng.integers(0, 4, n).astype(np.uint8)
        assert oracle.score(a, b, sc) == score_from_edit_distance(a, b, sc)


def test_score_bounds():
    rng = np.random.default_rng(5)
    for _ in range(200):
        m, n = rng.integers(0, 60, 2)
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = rng.integers(0, 4, n).astype(np.uint8)
        s = oracle.score(a, b, P)
        assert -max(m, n) <= s <= min(m, n) - abs(int(m) - int(n))


def test_metamorphic_invariants():
    rng = np.random.default_rng(6)
    for _ in range(60):
        m, n = rng.integers(0, 90, 2)
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = rng.integers(0, 4, n).astype(np.uint8)
        for sc in [P, (2, -3, -2)]:
            s, p = oracle.align(a, b, sc)
            # swap keeps the score
            assert oracle.score(b, a, sc) == s
            # reversing both keeps the score
            assert oracle.score(a[::-1].copy(), b[::-1].copy(), sc) == s
            # relabelling the alphabet keeps score and path
            perm = rng.permutation(4).astype(np.uint8)
            s2, p2 = oracle.align(perm[a], perm[b], sc)
            assert s2 == s and p2.tolist() == p.tolist()
            # appending a common symbol gains at least one match
            c = np.array([rng.integers(0, 4)], np.uint8)
            assert oracle.score(np.concatenate([a, c]), np.concatenate([b, c]), sc) >= s + sc[0]
            # the path consumes both sequences and rescores to s
            r, ok = oracle.rescore(p, a, b, sc)
            assert ok and r == s
            assert path_score(p.tolist(), a, b, sc) == s


def test_dirs_dump_matches_traceback():
    rng = np.random.default_rng(7)
    a = rng.integers(0, 4, 40).astype(np.uint8)
    b = rng.integers(0, 4, 33).astype(np.uint8)
    C = oracle.dirs(a, b, P)
    assert C[0, 0] == 0 and (C[1:, 0] == 2).all() and (C[0, 1:] == 3).all()
    s, p = oracle.align(a, b, P)
    i, j = len(a), len(b)
    for mv in p[::-1].tolist():
        assert C[i, j] == mv
        if mv == 1:
            i, j = i - 1, j - 1
        elif mv == 2:
            i -= 1
        else:
            j -= 1
    assert (i, j) == (0, 0)


def test_two_row_mode_matches_full_matrix():
    rng = np.random.default_rng(8)
    for _ in range(20):
        m, n = rng.integers(0, 200, 2)
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = rng.integers(0, 4, n).astype(np.uint8)
        s_full, p_full = oracle.align(a, b, P)
        s_two, p_two = oracle.align(a, b, P, full_limit_bytes=0)
        assert s_full == s_two and p_full.tolist() == p_two.tolist()


def test_batch_and_allpairs_structure():
    from workloads import config_batch, pack_pairs, config_allpairs, pack_seqs
    pairs = config_batch(seed=77, npairs=24, lo=10, hi=150)
    pool, ao, al, bo, bl = pack_pairs(pairs)
    scores, paths = oracle.align_batch(pool, ao, al, bo, bl, P)
    scores2, _ = oracle.align_batch(pool, ao, al, bo, bl, P, with_paths=False)
    for k in range(len(pairs)):
        s, p = oracle.align(pairs.a[k], pairs.b[k], P)
        assert scores[k] == s == scores2[k]
        assert paths[k].tolist() == p.tolist()
    seqs = config_allpairs(seed=78, nseq=12, lo=20, hi=90, root_len=200)
    pool, off, lens = pack_seqs(seqs)
    M = oracle.allpairs(pool, off, lens, P)
    assert (M == M.T).all()
    assert (np.diag(M) == lens * P[0]).all()
    for i in range(len(seqs)):
        for j in range(i + 1, len(seqs)):
            assert M[i, j] == oracle.score(seqs[i], seqs[j], P)
    # the number of off-diagonal pairs is n(n-1)/2 (paper Eq. 2)
    assert np.triu_indices(len(seqs), 1)[0].size == len(seqs) * (len(seqs) - 1) // 2


# ---------------------------------------------------------------------------
# band certificate
# ---------------------------------------------------------------------------

def test_u_out_bounds_every_path_leaving_the_band():
    rng = np.random.default_rng(9)
    for m in range(0, 7):
        for n in range(0, 7):
            for _ in range(2):
                a = rng.integers(0, 4, m).astype(np.uint8)
                b = rng.integers(0, 4, n).astype(np.uint8)
                for sc in [P, (2, -3, -2), (1, 0, -1)]:
                    for w in range(0, 7):
                        best_out = max_score_leaving_band(a, b, w, sc)
                        u = band.u_out(m, n, w, sc)
                        if u is None:
                            assert best_out is None
                        elif best_out is not None:
                            assert best_out <= u


def test_u_out_is_attained_for_matching_sequences():
    # all-match symbols make the bound tight: a path with exactly the minimum
    # number of gaps and only matches on the diagonal reaches U_out(w).
    for m, n, w in [(6, 6, 1), (6, 5, 0), (5, 6, 2), (6, 6, 0)]:
        a = np.zeros(m, np.uint8)
        b = np.zeros(n, np.uint8)
        assert max_score_leaving_band(a, b, w, P) == band.u_out(m, n, w, P)


def test_w_cert_and_w_path():
    rng = np.random.default_rng(10)
    for _ in range(300):
        m, n = rng.integers(0, 40, 2)
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = rng.integers(0, 4, n).astype(np.uint8)
        for sc in [P, (2, -3, -2)]:
            s, p = oracle.align(a, b, sc)
            wc = band.w_cert(s, m, n, sc)
            assert band.certifies(s, m, n, wc, sc)
            if wc > 0:
                assert not band.certifies(s, m, n, wc - 1, sc)
            # the tie-break path lies in the certified band
            assert band.w_path(p, m, n) <= wc
    # paper constants: w_cert = floor(K/3), K = min(m,n) - |m-n| - S
    for _ in range(200):
        m, n = rng.integers(1, 60, 2)
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = rng.integers(0, 4, n).astype(np.uint8)
        s = oracle.score(a, b, P)
        K = min(m, n) - abs(int(m) - int(n)) - s
        assert band.w_cert(s, m, n, P) == min(K // 3, min(m, n))


def test_band_cells_count():
    for m, n, w in [(5, 7, 1), (7, 5, 0), (10, 10, 3), (1, 9, 0)]:
        cnt = sum(1 for i in range(1, m + 1) for j in range(1, n + 1) if band.in_band(i, j, m, n, w))
        assert band.band_cells(m, n, w) == cnt
