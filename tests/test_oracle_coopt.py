"""Pins for the co-optimal alignment oracle (oracle/coopt.py, orc_count),
independent of its code:

* exhaustive enumeration of every alignment for m, n <= 6: the number of
  optimal ones, and the optimal ones themselves in the stated order;
* closed forms: with match = mismatch = 2*gap every alignment scores
  (m+n)*gap, so all D(m,n) (Delannoy) alignments are optimal -- past 2^64 this
  checks the flag and the count modulo 2^64; identical sequences under the
  paper's scoring have exactly one; an empty side has exactly one; a
  one-letter sequence against b has as many as b has copies of the letter
  (or len(b) if it has none);
* the first enumerated path is the oracle's tie-broken path, every path
  rescores to the optimum, and the paths are distinct.
"""
from math import comb

import numpy as np
import pytest

import oracle
from oracle import coopt
from pins import all_paths, brute_force_all
from workloads import mutate, random_seq

P = (1, -1, -1)


def delannoy(m, n):
    return sum(comb(m, k) * comb(n, k) * 2 ** k for k in range(min(m, n) + 1))


@pytest.mark.parametrize("alphabet", [2, 4])
def test_counts_and_order_by_exhaustive_enumeration(alphabet):
    rng = np.random.default_rng(70 + alphabet)
    for m in range(0, 7):
        for n in range(0, 7):
            reps = 2 if m * n >= 25 else 4
            for _ in range(reps):
                a = rng.integers(0, alphabet, m).astype(np.uint8)
                b = rng.integers(0, alphabet, n).astype(np.uint8)
                for sc in [P, (2, -3, -2), (1, 0, 0)]:
                    best, opt = brute_force_all(a, b, sc)
                    s, c = coopt.count_exact(a, b, sc)
                    assert (s, c) == (best, len(opt)), (a, b, sc)
                    assert coopt.count(a, b, sc) == (best, len(opt), False)
                    got = coopt.enumerate_paths(a, b, sc, k=len(opt) + 3)
                    assert [tuple(p.tolist()) for p in got] == opt, (a, b, sc)
                    few = coopt.enumerate_paths(a, b, sc, k=2)
                    assert [tuple(p.tolist()) for p in few] == opt[:2]


def test_delannoy_closed_form_and_overflow_flag():
    sc = (-2, -2, -1)
    rng = np.random.default_rng(5)
    assert len(all_paths(4, 5)) == delannoy(4, 5)
    # (30, 24), (44, 18): at the end cell the vertical neighbour's addition is
    # the first sum to reach 2^64; (14, 73), (15, 63), (16, 55): only the
    # horizontal neighbour has reached 2^64 and the sum does not wrap, so the
    # flag must come from that neighbour
    for m, n in [(0, 0), (0, 7), (3, 3), (6, 6), (20, 17), (35, 35), (41, 40), (60, 90), (200, 150),
                 (30, 24), (44, 18), (14, 73), (15, 63), (16, 55)]:
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = rng.integers(0, 4, n).astype(np.uint8)
        dmn = delannoy(m, n)
        s, c, f = coopt.count(a, b, sc)
        assert s == (m + n) * -1
        assert c == dmn % (1 << 64)
        assert f == (dmn >= (1 << 64)), (m, n)
        if m * n <= 60 * 90:
            assert coopt.count_exact(a, b, sc) == ((m + n) * -1, dmn)
    # the smallest square past 2^64 flips the flag exactly there
    k = next(k for k in range(1, 60) if delannoy(k, k) >= (1 << 64))
    z = np.zeros(k, np.uint8)
    assert coopt.count(z[:k - 1], z[:k - 1], sc)[2] is False
    assert coopt.count(z, z, sc)[2] is True


def test_identical_empty_and_single_letter():
    rng = np.random.default_rng(8)
    s = random_seq(rng, 300)
    assert coopt.count(s, s, P) == (300, 1, False)
    assert coopt.count(s[:0], s, P) == (-300, 1, False)
    assert coopt.count(s, s[:0], P) == (-300, 1, False)
    for _ in range(20):
        b = rng.integers(0, 4, int(rng.integers(1, 40))).astype(np.uint8)
        x = np.array([rng.integers(0, 4)], np.uint8)
        occ = int((b == x[0]).sum())
        assert coopt.count(x, b, P)[1] == (occ if occ else len(b)), (x, b)


def test_enumeration_on_related_pairs():
    rng = np.random.default_rng(9)
    for _ in range(6):
        a = random_seq(rng, int(rng.integers(40, 160)))
        b = mutate(rng, a, 0.2)
        s, c = coopt.count_exact(a, b, P)
        assert coopt.count(a, b, P) == (s, c % (1 << 64), c >= (1 << 64))
        paths = coopt.enumerate_paths(a, b, P, k=12)
        assert len(paths) == min(12, c)
        s0, p0 = oracle.align(a, b, P)
        assert s0 == s and paths[0].tolist() == p0.tolist()
        assert len({p.tobytes() for p in paths}) == len(paths)
        for p in paths:
            r, ok = oracle.rescore(p, a, b, P)
            assert ok and r == s


def test_batch_matches_single():
    rng = np.random.default_rng(10)
    pairs = []
    for _ in range(30):
        a = random_seq(rng, int(rng.integers(0, 120)))
        pairs.append((a, mutate(rng, a, 0.15)))
    pool = np.concatenate([np.concatenate([a, b]) for a, b in pairs])
    ao, al, bo, bl, o = [], [], [], [], 0
    for a, b in pairs:
        ao.append(o); al.append(len(a)); o += len(a)
        bo.append(o); bl.append(len(b)); o += len(b)
    s, c, f = coopt.count_batch(pool, ao, al, bo, bl, P)
    for k, (a, b) in enumerate(pairs):
        assert (int(s[k]), int(c[k]), bool(f[k])) == coopt.count(a, b, P)
