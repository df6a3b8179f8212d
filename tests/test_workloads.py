"""The seeded generators: determinism, shapes and the mutation model's rates."""
import numpy as np

from workloads import (config_allpairs, config_band_batch, config_batch, config_long_pair,
                       config_single, mutate, pack_pairs, pack_seqs, random_seq)


def test_determinism_and_alphabet():
    a1 = config_single(seed=5).a[0]
    a2 = config_single(seed=5).a[0]
    assert (a1 == a2).all() and a1.dtype == np.uint8 and a1.max() <= 3
    p = config_batch(seed=3, npairs=16)
    q = config_batch(seed=3, npairs=16)
    assert all((x == y).all() for x, y in zip(p.b, q.b))
    lens = [x.shape[0] for x in p.a]
    assert min(lens) >= 100 and max(lens) <= 2000


def test_mutation_rates():
    rng = np.random.default_rng(0)
    a = random_seq(rng, 200000)
    b = mutate(rng, a, 0.10)
    # expected length change: ins and del are equally likely, each adds/removes
    # ~2 bases (geometric(0.5) mean 2), so the lengths stay close
    assert abs(b.shape[0] - a.shape[0]) < 0.01 * a.shape[0]
    # zero rate is the identity
    assert (mutate(rng, a[:1000], 0.0) == a[:1000]).all()
    # substitution-only mutation keeps the length and changes ~rate of sites
    c = mutate(rng, a, 0.2, p_sub=1.0, p_ins=0.0)
    assert c.shape == a.shape
    frac = float((c != a).mean())
    assert 0.19 < frac < 0.21


def test_insertions_and_deletions_only():
    rng = np.random.default_rng(1)
    a = random_seq(rng, 100000)
    ins = mutate(rng, a, 0.05, p_sub=0.0, p_ins=1.0)
    assert ins.shape[0] > a.shape[0]
    # every ancestral base survives in order
    dele = mutate(rng, a, 0.05, p_sub=0.0, p_ins=0.0)
    assert dele.shape[0] < a.shape[0]
    # ~5% of sites start a deletion of mean length 2 (overlaps merge)
    assert 0.88 * a.shape[0] < dele.shape[0] < 0.92 * a.shape[0]


def test_packing():
    p = config_batch(seed=9, npairs=5, lo=10, hi=20)
    pool, ao, al, bo, bl = pack_pairs(p)
    for k in range(5):
        assert (pool[ao[k]:ao[k] + al[k]] == p.a[k]).all()
        assert (pool[bo[k]:bo[k] + bl[k]] == p.b[k]).all()
    seqs = config_allpairs(seed=1, nseq=10, lo=50, hi=100, root_len=300)
    pool, off, lens = pack_seqs(seqs)
    assert lens.min() >= 50 and lens.max() <= 100
    assert all((pool[off[k]:off[k] + lens[k]] == seqs[k]).all() for k in range(10))


def test_long_pair_and_band_batch_shapes():
    lp = config_long_pair(length=4096)
    assert lp.a[0].shape[0] == 4096 and abs(lp.b[0].shape[0] - 4096) < 200
    bb = config_band_batch(npairs=6, lo=1000, hi=1500)
    assert len(bb) == 6 and all(1000 <= x.shape[0] <= 1500 for x in bb.a)
