"""Any byte is a legal symbol: the recurrence compares symbols for equality
only (a match or a mismatch), so every entry point must agree with the
oracle, which compares whole bytes, whatever the alphabet.

Pairs whose bytes take at most four values that one two-bit field tells
apart (nucleotide codes 0..3, the letters ACGT or acgu, bytes 252..255) are
swept with those two bits as codes; any other pair (five or more distinct
bytes, or four no two-bit field separates, such as 1, 2, 4, 8) is swept by
comparing bytes.  Both kinds are mixed in one batch here, so each launch
serves both parts of its queue."""
import numpy as np
import pytest

import oracle
from oracle import coopt
from oracle import msa as omsa
from workloads import Pairs, pack_pairs, pack_seqs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2412_21103_amd as nwp  # noqa: E402
from gpu_util import gpu_align, gpu_allpairs, gpu_batch, say  # noqa: E402

P = (1, -1, -1)
ALPHABETS = {
    "codes": bytes([0, 1, 2, 3]),
    "ACGT": b"ACGT",
    "acgu": b"acgu",
    "high": bytes([252, 253, 254, 255]),
    "bits": bytes([1, 2, 4, 8]),
    "ACGTN": b"ACGTN",
    "protein": b"ACDEFGHIKLMNPQRSTVWY",
    "bytes": bytes(range(256)),
}


def seq(rng, n, alpha):
    a = np.frombuffer(alpha, np.uint8)
    return a[rng.integers(0, len(a), int(n))].copy()


def mutated(rng, s, alpha, rate):
    """Substitutions (by a different symbol of the alphabet), insertions and
    deletions at `rate` per site, 70/15/15."""
    a = np.frombuffer(alpha, np.uint8)
    out = []
    for x in s.tolist():
        u = rng.random()
        if u >= rate:
            out.append(x)
        elif u < 0.7 * rate:
            choices = a[a != x]
            out.append(int(choices[rng.integers(len(choices))]) if len(choices) else x)
        elif u < 0.85 * rate:
            out.append(x)
            out.extend(a[rng.integers(0, len(a), 1 + int(rng.geometric(0.5)) - 1)].tolist())
        # else: deleted
    return np.array(out, np.uint8)


def _dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")


def _mixed_pairs(seed, npairs, hi):
    rng = np.random.default_rng(seed)
    names = list(ALPHABETS)
    A, B, tags = [], [], []
    for k in range(npairs):
        name = names[k % len(names)]
        a = seq(rng, int(rng.integers(0, hi)), ALPHABETS[name])
        A.append(a)
        B.append(mutated(rng, a, ALPHABETS[name], float(rng.uniform(0.02, 0.3))))
        tags.append(name)
    return Pairs(A, B, "alphabets"), tags


@pytest.mark.parametrize("name", list(ALPHABETS))
def test_single_pairs_any_alphabet(name):
    rng = np.random.default_rng(sum(name.encode()))
    alpha = ALPHABETS[name]
    # one-wave engine below 512 columns, multi-wave engine above
    for m in (57, 300, 1500):
        a = seq(rng, m, alpha)
        b = mutated(rng, a, alpha, 0.15)
        say(f"alphabet {name}: {len(a)} x {len(b)}")
        for sc in (P, (2, -3, -2)):
            s_ref, p_ref = oracle.align(a, b, sc)
            s, p = gpu_align(a, b, sc)
            assert s == s_ref, (name, m, sc, s, s_ref)
            assert p.tolist() == p_ref.tolist(), (name, m, sc)
            s2, _ = gpu_align(a, b, sc, score_only=True)
            assert s2 == s_ref, (name, m, sc)


def test_unrelated_bytes_long_pair():
    # two independent sequences over all 256 bytes on the multi-wave engine
    rng = np.random.default_rng(9)
    a, b = seq(rng, 2500, ALPHABETS["bytes"]), seq(rng, 2300, ALPHABETS["bytes"])
    s_ref, p_ref = oracle.align(a, b, P)
    s, p = gpu_align(a, b, P)
    assert s == s_ref and p.tolist() == p_ref.tolist()


def test_batch_mixed_alphabets():
    pairs, tags = _mixed_pairs(3, 96, 900)
    pool, ao, al, bo, bl = pack_pairs(pairs)
    ml = int(max(al.max(), bl.max()))
    say("alphabets: mixed batch")
    s_ref, p_ref = oracle.align_batch(pool, ao, al, bo, bl, P)
    s, paths, plen = gpu_batch(pool, ao, al, bo, bl, ml, P)
    bad = np.nonzero(s != s_ref)[0]
    assert len(bad) == 0, [(int(k), tags[k]) for k in bad[:8]]
    for k in range(len(pairs)):
        assert paths[k].tolist() == p_ref[k].tolist(), (k, tags[k])
    s2, _ = gpu_batch(pool, ao, al, bo, bl, ml, P, score_only=True)
    assert (s2 == s_ref).all()


@pytest.mark.parametrize("w0,doubling", [(0, False), (16, False), (4, True)])
def test_banded_mixed_alphabets(w0, doubling):
    pairs, tags = _mixed_pairs(4, 64, 1200)
    pool, ao, al, bo, bl = pack_pairs(pairs)
    ml = int(max(al.max(), bl.max()))
    say(f"alphabets: banded from {w0}, doubling {doubling}")
    s_ref, p_ref = oracle.align_batch(pool, ao, al, bo, bl, P)
    out = nwp.align_batch_banded(_dev(pool, np.uint8), _dev(ao, np.int64), _dev(al, np.int32), _dev(bo, np.int64),
                                 _dev(bl, np.int32), ml, P, w_default=w0, doubling=doubling)
    torch.cuda.synchronize()
    s, paths, poff, plen = (t.cpu().numpy() for t in out[:4])
    for k in range(len(pairs)):
        assert s[k] == s_ref[k], (k, tags[k])
        assert paths[poff[k]:poff[k] + plen[k]].tolist() == p_ref[k].tolist(), (k, tags[k])


def test_allpairs_mixed_alphabets():
    rng = np.random.default_rng(5)
    seqs = []
    for k, name in enumerate(list(ALPHABETS) * 3):
        seqs.append(seq(rng, int(rng.integers(0, 400)), ALPHABETS[name]))
    pool, off, lens = pack_seqs(seqs)
    say("alphabets: all-pairs")
    M = gpu_allpairs(pool, off, lens, int(lens.max()), P)
    assert np.array_equal(M, oracle.allpairs(pool, off, lens, P))


def test_cooptimal_mixed_alphabets():
    pairs, tags = _mixed_pairs(6, 40, 160)
    pool, ao, al, bo, bl = pack_pairs(pairs)
    ml = max(1, int(max(al.max(), bl.max())))
    say("alphabets: co-optimal counts and paths")
    d = [_dev(pool, np.uint8), _dev(ao, np.int64), _dev(al, np.int32), _dev(bo, np.int64), _dev(bl, np.int32)]
    out = nwp.cooptimal(*d, ml, P, k=3)
    torch.cuda.synchronize()
    scores, counts, sat, paths, poff, plen, npaths = (o.cpu().numpy() for o in out)
    counts = counts.view(np.uint64)
    s_ref, c_ref, f_ref = coopt.count_batch(pool, ao, al, bo, bl, P)
    assert np.array_equal(scores, s_ref)
    assert np.array_equal(counts, c_ref)
    assert np.array_equal(sat, f_ref)
    for q, (a, b) in enumerate(zip(pairs.a, pairs.b)):
        ref = coopt.enumerate_paths(a, b, P, k=3)
        assert npaths[q] == len(ref), (q, tags[q])
        cap = len(a) + len(b)
        for r, pr in enumerate(ref):
            assert paths[poff[q] + r * cap: poff[q] + r * cap + plen[q, r]].tolist() == pr.tolist(), (q, r)


def test_center_star_letters():
    # a family written in letters, with '-' as the gap byte
    rng = np.random.default_rng(8)
    root = seq(rng, 700, b"ACGT")
    seqs = [mutated(rng, root, b"ACGT", float(rng.uniform(0.02, 0.2)))[: int(rng.integers(300, 700))].copy()
            for _ in range(12)]
    pool, off, lens = pack_seqs(seqs)
    ml = int(lens.max())
    dp, do, dl = _dev(pool, np.uint8), _dev(off, np.int64), _dev(lens, np.int32)
    S = nwp.allpairs(dp, do, dl, ml, P)
    c, M, w = nwp.center_star(dp, do, dl, ml, S, P, gap_byte=ord("-"))
    torch.cuda.synchronize()
    c_ref, M_ref = omsa.center_star(seqs, P, gap_byte=ord("-"), scores=S.cpu().numpy())
    assert int(c.item()) == c_ref
    w = int(w.item())
    assert w == M_ref.shape[1]
    assert np.array_equal(M.cpu().numpy()[:, :w], M_ref)
