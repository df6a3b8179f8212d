"""Co-optimal alignments on the GPU against the oracle (oracle/coopt.py):
scores, counts modulo 2^64 and the >= 2^64 flag bit for bit, and the first k
paths byte for byte, on ragged strips, empty sides, all-tied scorings whose
counts pass 2^64, skipped pairs, and the full 4096-pair batch workload."""
from math import comb

import numpy as np
import pytest

import oracle
from oracle import coopt
from workloads import Pairs, config_batch, mutate, pack_pairs, random_seq

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2412_21103_amd as nwp  # noqa: E402
from gpu_util import say  # noqa: E402

P = (1, -1, -1)
TIED = (-2, -2, -1)  # every alignment scores (m+n)*gap: all Delannoy(m,n) are optimal


def delannoy(m, n):
    return sum(comb(m, k) * comb(n, k) * 2 ** k for k in range(min(m, n) + 1))


def _dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")


def _run(pairs, scoring=P, k=0, max_len=None):
    if not isinstance(pairs, Pairs):
        pairs = Pairs([a for a, _ in pairs], [b for _, b in pairs], "cooptimal")
    pool, ao, al, bo, bl = pack_pairs(pairs)
    if max_len is None:
        max_len = max(1, int(max(al.max(initial=0), bl.max(initial=0))))
    d = [_dev(pool if len(pool) else np.zeros(1, np.uint8), np.uint8), _dev(ao, np.int64), _dev(al, np.int32),
         _dev(bo, np.int64), _dev(bl, np.int32)]
    out = nwp.cooptimal(*d, max_len, scoring, k=k)
    torch.cuda.synchronize()
    res = [o.cpu().numpy() for o in out]
    res[1] = res[1].view(np.uint64)
    return (pool, ao, al, bo, bl), res


def _check_counts(packed, res, scoring):
    s_ref, c_ref, f_ref = coopt.count_batch(*packed, scoring)
    assert np.array_equal(res[0], s_ref)
    assert np.array_equal(res[1], c_ref)
    assert np.array_equal(res[2], f_ref)


@pytest.mark.parametrize("scoring", [P, (2, -3, -2), (1, 0, -1), (3, -1, -2)])
def test_counts_match_oracle(scoring):
    rng = np.random.default_rng(40)
    pairs = []
    for n in [1, 2, 63, 64, 65, 127, 128, 129, 200, 255, 256, 257, 300]:
        a = random_seq(rng, int(rng.integers(1, 320)))
        pairs.append((a, mutate(rng, random_seq(rng, n), 0.1)[:n].copy()))
    for _ in range(40):
        a = random_seq(rng, int(rng.integers(0, 400)))
        pairs.append((a, mutate(rng, a, float(rng.uniform(0.0, 0.3)))))
    pairs += [(random_seq(rng, 0), random_seq(rng, 9)), (random_seq(rng, 7), random_seq(rng, 0)),
              (random_seq(rng, 0), random_seq(rng, 0))]
    say(f"cooptimal counts: {len(pairs)} pairs, scoring {scoring}")
    packed, res = _run(pairs, scoring)
    _check_counts(packed, res, scoring)


def test_counts_past_two_to_the_64():
    rng = np.random.default_rng(41)
    pairs = []
    for m, n in [(5, 5), (30, 30), (36, 36), (40, 41), (64, 64), (130, 90), (200, 260), (1, 300), (300, 1)]:
        pairs.append((rng.integers(0, 4, m).astype(np.uint8), rng.integers(0, 4, n).astype(np.uint8)))
    say("cooptimal counts: all-tied scoring, counts past 2^64")
    packed, res = _run(pairs, TIED)
    _check_counts(packed, res, TIED)
    want = [delannoy(len(a), len(b)) for a, b in pairs]
    assert res[1].tolist() == [d % (1 << 64) for d in want]
    assert res[2].tolist() == [int(d >= (1 << 64)) for d in want]
    assert 0 < sum(res[2].tolist()) < len(pairs)


def test_skipped_pairs_and_max_len():
    rng = np.random.default_rng(42)
    pairs = [(random_seq(rng, 100), random_seq(rng, 90)), (random_seq(rng, 150), random_seq(rng, 40)),
             (random_seq(rng, 30), random_seq(rng, 151))]
    packed, res = _run(pairs, P, k=2, max_len=120)
    s_ref, c_ref, f_ref = coopt.count_batch(*packed, P)
    assert res[0][0] == s_ref[0] and res[1][0] == c_ref[0]
    assert res[0][1] == np.iinfo(np.int32).min and res[0][2] == np.iinfo(np.int32).min
    assert res[1][1:].tolist() == [0, 0] and res[6][1:].tolist() == [0, 0]


@pytest.mark.parametrize("scoring,k", [(P, 6), ((1, 0, -1), 9), ((2, -3, -2), 3)])
def test_enumeration_matches_oracle(scoring, k):
    rng = np.random.default_rng(43)
    pairs = []
    for _ in range(24):
        a = random_seq(rng, int(rng.integers(0, 180)))
        pairs.append((a, mutate(rng, a, float(rng.uniform(0.05, 0.35)))))
    pairs.append((random_seq(rng, 0), random_seq(rng, 5)))
    pairs.append((random_seq(rng, 4), random_seq(rng, 0)))
    say(f"cooptimal paths: {len(pairs)} pairs, k={k}, scoring {scoring}")
    packed, res = _run(pairs, scoring, k=k)
    _check_counts(packed, res, scoring)
    scores, counts, sat, paths, poff, plen, npaths = res
    for q, (a, b) in enumerate(pairs):
        ref = coopt.enumerate_paths(a, b, scoring, k=k)
        assert npaths[q] == len(ref), q
        cap = len(a) + len(b)
        for r, pr in enumerate(ref):
            got = paths[poff[q] + r * cap: poff[q] + r * cap + plen[q, r]]
            assert got.tolist() == pr.tolist(), (q, r)


def test_enumeration_all_tied_small():
    rng = np.random.default_rng(44)
    pairs = [(rng.integers(0, 4, m).astype(np.uint8), rng.integers(0, 4, n).astype(np.uint8))
             for m, n in [(3, 4), (4, 4), (6, 5), (70, 3), (2, 140)]]
    packed, res = _run(pairs, TIED, k=40)
    _check_counts(packed, res, TIED)
    paths, poff, plen, npaths = res[3:]
    for q, (a, b) in enumerate(pairs):
        ref = coopt.enumerate_paths(a, b, TIED, k=40)
        assert npaths[q] == len(ref)
        cap = len(a) + len(b)
        for r, pr in enumerate(ref):
            assert paths[poff[q] + r * cap: poff[q] + r * cap + plen[q, r]].tolist() == pr.tolist(), (q, r)


def test_first_path_is_the_batch_path():
    rng = np.random.default_rng(45)
    pairs = []
    for _ in range(16):
        a = random_seq(rng, int(rng.integers(100, 700)))
        pairs.append((a, mutate(rng, a, 0.12)))
    packed, res = _run(pairs, P, k=1)
    s_ref, p_ref = oracle.align_batch(*packed, P)
    assert np.array_equal(res[0], s_ref)
    paths, poff, plen = res[3], res[4], res[5]
    for q in range(len(pairs)):
        assert paths[poff[q]: poff[q] + plen[q, 0]].tolist() == p_ref[q].tolist()


def test_batch_workload_full_size():
    pairs = config_batch()
    say(f"cooptimal counts at full size: {len(pairs)} pairs")
    packed, res = _run(pairs, P)
    _check_counts(packed, res, P)


def test_team_shapes():
    """Pairs of 2^16 cells or more are filled by the four waves of a block:
    skinny and wide pairs (one to three strips), ragged last strips, and
    pairs just below and above that size, mixed with single-wave pairs."""
    rng = np.random.default_rng(46)
    shapes = [(3000, 60), (60, 3000), (1500, 130), (700, 700), (256, 257), (255, 256), (1030, 1), (1, 1030),
              (400, 513), (513, 400), (2100, 129), (90, 90), (300, 5)]
    pairs = []
    for m, n in shapes:
        a = random_seq(rng, m)
        b = mutate(rng, a, 0.1)[:n].copy() if n <= m else random_seq(rng, n)
        if len(b) < n:
            b = np.concatenate([b, random_seq(rng, n - len(b))])
        pairs.append((a, b))
    for sc in (P, TIED):
        say(f"cooptimal team shapes, scoring {sc}")
        packed, res = _run(pairs, sc)
        _check_counts(packed, res, sc)
