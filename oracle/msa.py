"""Center-star multiple alignment: CPU reference (TEST INFRASTRUCTURE ONLY).

The paper's multiple-alignment extension (Sec. 3.2, Multiple Alignment):
choose a center sequence from the all-pairs scoring matrix, align
every other sequence to the center, then merge the pairwise alignments one
after another, using the aligned center as the reference.  The paper leaves
the details open; the readings taken here are:

* the center maximises the sum of its scores against the other sequences
  (its row of the score matrix without the diagonal); ties go to the lowest
  index;
* each pairwise alignment puts the center in the rows (a) and the other
  sequence in the columns (b), with the single-path traceback of ``align``
  (D > U > L);
* merging keeps every gap already in the growing alignment ("once a gap,
  always a gap"): walking the merged center row and the new pairwise
  alignment side by side, an insertion of the new alignment fills an existing
  insertion column of the merged alignment if one is free at that point, and
  otherwise opens a new column (a gap in every row merged so far); a free
  existing insertion column gets a gap in the new row.  Rows are kept in the
  input order, the center's own row included.  The gap byte must not occur
  in the sequences.

Everything here is plain Python over the oracle's own pairwise alignments, in
the order the paper describes.
"""
from __future__ import annotations

import numpy as np

from . import PAPER_SCORING, D, U, L, align, allpairs


def center_index(scores: np.ndarray) -> int:
    """Index of the row with the largest off-diagonal sum (lowest on ties)."""
    S = np.asarray(scores, dtype=np.int64)
    sums = S.sum(axis=1) - np.diag(S)
    return int(np.argmax(sums))


def pairwise_to_center(seqs, c: int, scoring=PAPER_SCORING):
    """Forward move strings aligning the center (rows) with every sequence k."""
    return {k: align(seqs[c], seqs[k], scoring)[1] for k in range(len(seqs)) if k != c}


def merge(seqs, c: int, paths, gap_byte: int, order=None) -> np.ndarray:
    """Merge the pairwise alignments to the center, in index order (or in
    ``order``), into one multiple alignment (rows in input order).
    ``paths[k]`` aligns seqs[c] (rows) with seqs[k] (columns)."""
    center = [int(x) for x in seqs[c]]
    # the merged alignment: the center row (ints, None for a gap) and the rows
    # merged so far, column by column
    cen_row = list(center)
    rows = {}
    for k in (sorted(paths) if order is None else order):
        seq = [int(x) for x in seqs[k]]
        path = [int(x) for x in paths[k]]
        new_cen, new_rows, new_k = [], {r: [] for r in rows}, []
        col = 0   # column of the merged alignment
        p = 0     # move of the pairwise alignment
        j = 0     # next residue of seqs[k]
        while col < len(cen_row) or p < len(path):
            here_gap = col < len(cen_row) and cen_row[col] is None
            ins = p < len(path) and path[p] == L
            if here_gap and ins:          # insertion meets a free insertion column
                new_cen.append(None)
                for r in rows:
                    new_rows[r].append(rows[r][col])
                new_k.append(seq[j])
                j += 1
                col += 1
                p += 1
            elif here_gap:                # insertion column of earlier rows only
                new_cen.append(None)
                for r in rows:
                    new_rows[r].append(rows[r][col])
                new_k.append(None)
                col += 1
            elif ins:                     # a new insertion column
                new_cen.append(None)
                for r in rows:
                    new_rows[r].append(None)
                new_k.append(seq[j])
                j += 1
                p += 1
            else:                         # a center residue: D or U
                mv = path[p]
                new_cen.append(cen_row[col])
                for r in rows:
                    new_rows[r].append(rows[r][col])
                if mv == D:
                    new_k.append(seq[j])
                    j += 1
                else:
                    assert mv == U
                    new_k.append(None)
                col += 1
                p += 1
        assert j == len(seq)
        cen_row = new_cen
        rows = new_rows
        rows[k] = new_k
    width = len(cen_row)
    out = np.full((len(seqs), width), gap_byte, dtype=np.uint8)
    rows[c] = cen_row
    for r, row in rows.items():
        for x, v in enumerate(row):
            if v is not None:
                out[r, x] = v
    return out


def center_star(seqs, scoring=PAPER_SCORING, gap_byte: int = 255, scores=None):
    """Returns ``(center, msa)``: msa is uint8[nseq, width], gaps = gap_byte."""
    seqs = [np.asarray(s, dtype=np.uint8) for s in seqs]
    if scores is None:
        lens = np.array([len(s) for s in seqs], np.int32)
        off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
        pool = np.concatenate(seqs) if seqs else np.zeros(0, np.uint8)
        scores = allpairs(pool, off, lens, scoring)
    c = center_index(scores)
    return c, merge(seqs, c, pairwise_to_center(seqs, c, scoring), gap_byte)
