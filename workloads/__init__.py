"""Seeded synthetic workloads for the Needleman-Wunsch hot path.

This module only draws random sequences: it holds no alignment arithmetic and
is shared, unchanged, by the CPU oracle tests and the HIP path.  Sequences are
nucleotide codes 0..3 (A, C, G, T) stored as uint8.

The paper aligns real gene pairs (COL1A1 and THAP11, mouse against human, in its
strong-scaling analysis); those sequences are not available here, so seeded
random ancestors with a seeded point/indel mutation model stand in for them.

Mutation model (one pass over the ancestor, left to right, all draws vectorised
per sequence, in this order):

1. ``u = rng.random(L)``       -- site ``p`` carries an event iff ``u[p] < rate``.
2. ``kind = rng.random(L)``    -- event type: substitution if ``kind < p_sub``,
   insertion if ``kind < p_sub + p_ins``, deletion otherwise.
3. ``shift = rng.integers(1, 4, L)`` -- a substitution replaces base ``x`` by
   ``(x + shift) % 4`` (uniform over the three other bases).
4. ``k = rng.geometric(0.5, L)``  -- indel length, support >= 1.
5. inserted bases: ``rng.integers(0, 4, total_inserted)``.

A deletion at ``p`` removes sites ``p .. p+k-1`` (clipped at the end);
overlapping deletions remove the union of their spans, and substitutions or
insertions drawn at a removed site are discarded.  An insertion keeps its site
base unchanged and appends ``k`` random bases after it.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "random_seq",
    "mutate",
    "Pairs",
    "config_single",
    "config_long_pair",
    "config_batch",
    "config_allpairs",
    "config_band_batch",
    "pack_pairs",
    "pack_seqs",
]


def random_seq(rng: np.random.Generator, length: int) -> np.ndarray:
    """Uniform i.i.d. ACGT codes."""
    return rng.integers(0, 4, size=int(length), dtype=np.uint8)


def mutate(rng: np.random.Generator, seq: np.ndarray, rate: float,
           p_sub: float = 0.70, p_ins: float = 0.15) -> np.ndarray:
    """Return a mutated copy of ``seq`` (see the module docstring)."""
    seq = np.asarray(seq, dtype=np.uint8)
    L = seq.shape[0]
    if L == 0:
        return seq.copy()
    u = rng.random(L)
    kind = rng.random(L)
    shift = rng.integers(1, 4, size=L)
    k = rng.geometric(0.5, size=L)
    event = u < rate
    is_sub = event & (kind < p_sub)
    is_ins = event & (kind >= p_sub) & (kind < p_sub + p_ins)
    is_del = event & (kind >= p_sub + p_ins)

    # union of deletion spans [p, p+k) via a coverage count
    cover = np.zeros(L + 1, dtype=np.int64)
    dpos = np.nonzero(is_del)[0]
    np.add.at(cover, dpos, 1)
    np.add.at(cover, np.minimum(dpos + k[dpos], L), -1)
    removed = np.cumsum(cover[:L]) > 0

    out_base = seq.copy()
    out_base[is_sub] = ((seq[is_sub].astype(np.int64) + shift[is_sub]) % 4).astype(np.uint8)
    keep = ~removed
    ins_here = np.where(is_ins & keep, k, 0)
    reps = keep.astype(np.int64) + ins_here
    total = int(reps.sum())
    n_ins = int(ins_here.sum())
    ins_bases = rng.integers(0, 4, size=n_ins, dtype=np.uint8)

    out = np.empty(total, dtype=np.uint8)
    # position of each kept site in the output
    starts = np.cumsum(reps) - reps
    kept_idx = np.nonzero(keep)[0]
    out[starts[kept_idx]] = out_base[kept_idx]
    # inserted bases follow their site
    ins_sites = np.nonzero(ins_here)[0]
    if n_ins:
        lens = ins_here[ins_sites]
        first = starts[ins_sites] + 1
        # expand [first, first+len) ranges
        rel = np.arange(n_ins) - np.repeat(np.cumsum(lens) - lens, lens)
        out[np.repeat(first, lens) + rel] = ins_bases
    return out


class Pairs:
    """A list of (a, b) pairs plus metadata."""

    def __init__(self, a_list, b_list, name: str, meta=None):
        self.a = [np.asarray(x, dtype=np.uint8) for x in a_list]
        self.b = [np.asarray(x, dtype=np.uint8) for x in b_list]
        self.name = name
        self.meta = meta or {}

    def __len__(self):
        return len(self.a)

    def cells(self) -> int:
        return int(sum(int(x.shape[0]) * int(y.shape[0]) for x, y in zip(self.a, self.b)))


def pack_pairs(pairs: "Pairs"):
    """Concatenate all sequences into one pool.

    Returns ``pool (uint8), a_off (int64), a_len (int32), b_off (int64), b_len (int32)``.
    """
    lens = []
    for x, y in zip(pairs.a, pairs.b):
        lens.append(x.shape[0])
        lens.append(y.shape[0])
    lens = np.asarray(lens, dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    pool = np.concatenate([s for xy in zip(pairs.a, pairs.b) for s in xy]) if len(pairs) else np.zeros(0, np.uint8)
    a_off = offs[0::2].copy()
    b_off = offs[1::2].copy()
    a_len = lens[0::2].astype(np.int32)
    b_len = lens[1::2].astype(np.int32)
    return pool.astype(np.uint8), a_off, a_len, b_off, b_len


def pack_seqs(seqs):
    """Concatenate sequences: returns ``pool, off (int64), len (int32)``."""
    lens = np.asarray([s.shape[0] for s in seqs], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    pool = np.concatenate(seqs) if seqs else np.zeros(0, np.uint8)
    return pool.astype(np.uint8), offs, lens.astype(np.int32)


# ---------------------------------------------------------------------------
# The five workloads.  seed = 1000 * k for workload k unless given.
# ---------------------------------------------------------------------------

def config_single(seed: int = 1000, length: int = 1024) -> Pairs:
    """Two independent uniform-random sequences of equal length."""
    rng = np.random.default_rng(seed)
    a = random_seq(rng, length)
    b = random_seq(rng, length)
    return Pairs([a], [b], f"single_{length}", {"seed": seed})


def config_long_pair(seed: int = 2000, length: int = 65536, rate: float = 0.10) -> Pairs:
    """Ancestor of ``length`` bases and a 10%-mutated descendant (70/15/15)."""
    rng = np.random.default_rng(seed)
    a = random_seq(rng, length)
    b = mutate(rng, a, rate)
    return Pairs([a], [b], f"long_pair_{length}", {"seed": seed, "rate": rate})


def config_batch(seed: int = 3000, npairs: int = 4096, lo: int = 100, hi: int = 2000,
                 rate_lo: float = 0.05, rate_hi: float = 0.15) -> Pairs:
    """``npairs`` pairs: m ~ U{lo..hi}, b = mutate(a, r ~ U[rate_lo, rate_hi])."""
    rng = np.random.default_rng(seed)
    m = rng.integers(lo, hi + 1, size=npairs)
    rates = rng.uniform(rate_lo, rate_hi, size=npairs)
    A, B = [], []
    for k in range(npairs):
        a = random_seq(rng, m[k])
        A.append(a)
        B.append(mutate(rng, a, rates[k]))
    return Pairs(A, B, f"batch_{npairs}", {"seed": seed})


def config_allpairs(seed: int = 4000, nseq: int = 512, lo: int = 500, hi: int = 5000,
                    nroots: int = 8, root_len: int = 8000,
                    div_lo: float = 0.02, div_hi: float = 0.25):
    """``nseq`` descendants of ``nroots`` random roots, cut to lengths U{lo..hi}.

    Sequence k descends from root ``k % nroots`` with divergence U[div_lo, div_hi]
    (70/15/15 event mix) and is then cut to its first ``L_k`` bases.  If the
    mutated root is shorter than ``L_k`` it is kept whole.
    """
    rng = np.random.default_rng(seed)
    roots = [random_seq(rng, root_len) for _ in range(nroots)]
    lengths = rng.integers(lo, hi + 1, size=nseq)
    divs = rng.uniform(div_lo, div_hi, size=nseq)
    seqs = []
    for k in range(nseq):
        d = mutate(rng, roots[k % nroots], divs[k])
        seqs.append(d[: lengths[k]].copy())
    return seqs


def config_band_batch(seed: int = 5000, npairs: int = 8192, lo: int = 1000, hi: int = 20000,
                      div_lo: float = 0.01, div_hi: float = 0.30,
                      indel_lo: float = 0.05, indel_hi: float = 0.50) -> Pairs:
    """Learned-band workload: m ~ U{lo..hi}, divergence and indel fraction uniform.

    The indel fraction ``f`` of the mutation events is split evenly between
    insertions and deletions; substitutions take ``1 - f``.
    """
    rng = np.random.default_rng(seed)
    m = rng.integers(lo, hi + 1, size=npairs)
    div = rng.uniform(div_lo, div_hi, size=npairs)
    fr = rng.uniform(indel_lo, indel_hi, size=npairs)
    A, B = [], []
    for k in range(npairs):
        a = random_seq(rng, m[k])
        A.append(a)
        B.append(mutate(rng, a, div[k], p_sub=1.0 - fr[k], p_ins=fr[k] / 2.0))
    return Pairs(A, B, f"band_batch_{npairs}", {"seed": seed, "div": div, "indel_frac": fr})
