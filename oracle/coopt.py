"""Co-optimal alignments: CPU reference (TEST INFRASTRUCTURE ONLY).

Sec. 2.4 keeps every path from the bottom-right cell back to the origin that
reaches the optimal score.  Two questions about that set are answered here:

* how many such paths a pair has.  N(i,j), the number of optimal paths from
  (0,0) to (i,j), is 1 on the first row and column and elsewhere the sum of N
  over the neighbours whose candidate (Eq. 1 read as in R1: diagonal + s,
  vertical + g, horizontal + g) equals H(i,j).  ``count_exact`` keeps Python
  integers (small cases); ``count`` and ``count_batch`` call the C oracle,
  which keeps the count modulo 2^64 with a flag for "the true count is at
  least 2^64".
* the first k of them, in the order a depth-first search from (m,n) meets
  them when it tries the diagonal, then the vertical, then the horizontal
  move at every cell.  The first is the single tie-broken path of
  ``oracle.align``; equivalently the paths come in decreasing order of their
  reversed move strings under D > U > L.  Every cell such a search enters
  has an optimal move (or is the origin), so it never backtracks out of a
  dead end.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import PAPER_SCORING, D, L, U, _i32p, _i64p, _ptr, _u8, _u8p, fill, lib

_u64p = ctypes.POINTER(ctypes.c_uint64)
_bound = False


def _lib():
    global _bound
    L_ = lib()
    if not _bound:
        L_.orc_count.argtypes = [_u8p, ctypes.c_int64, _u8p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32, _i32p, _u64p, _u8p]
        L_.orc_count.restype = ctypes.c_int
        L_.orc_count_batch.argtypes = [ctypes.c_int32, _u8p, _i64p, _i32p, _i64p, _i32p, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, _i32p, _u64p, _u8p, ctypes.c_int32]
        L_.orc_count_batch.restype = ctypes.c_int
        _bound = True
    return L_


def count_exact(a, b, scoring=PAPER_SCORING):
    """``(score, N)`` with N an exact Python integer; plain loops, small inputs."""
    match, mismatch, gap = scoring
    a = [int(x) for x in a]
    b = [int(x) for x in b]
    m, n = len(a), len(b)
    H = [[0] * (n + 1) for _ in range(m + 1)]
    N = [[0] * (n + 1) for _ in range(m + 1)]
    for j in range(n + 1):
        H[0][j] = j * gap
        N[0][j] = 1
    for i in range(1, m + 1):
        H[i][0] = i * gap
        N[i][0] = 1
        for j in range(1, n + 1):
            d = H[i - 1][j - 1] + (match if a[i - 1] == b[j - 1] else mismatch)
            u = H[i - 1][j] + gap
            l_ = H[i][j - 1] + gap
            h = max(d, u, l_)
            H[i][j] = h
            N[i][j] = (N[i - 1][j - 1] if d == h else 0) + (N[i - 1][j] if u == h else 0) \
                + (N[i][j - 1] if l_ == h else 0)
    return H[m][n], N[m][n]


def count(a, b, scoring=PAPER_SCORING):
    """``(score, N mod 2^64, N >= 2^64)`` from the C oracle."""
    a, pa = _u8(a)
    b, pb = _u8(b)
    s = ctypes.c_int32(0)
    c = ctypes.c_uint64(0)
    f = ctypes.c_uint8(0)
    if _lib().orc_count(pa, a.shape[0], pb, b.shape[0], *scoring, ctypes.byref(s), ctypes.byref(c),
                        ctypes.byref(f)) < 0:
        raise MemoryError("oracle: out of host memory")
    return int(s.value), int(c.value), bool(f.value)


def count_batch(pool, a_off, a_len, b_off, b_len, scoring=PAPER_SCORING, nthreads: int = 0):
    """Scores (int32), counts mod 2^64 (uint64) and saturation flags (uint8)."""
    pool, pp = _u8(pool)
    a_off = np.ascontiguousarray(a_off, np.int64)
    b_off = np.ascontiguousarray(b_off, np.int64)
    a_len = np.ascontiguousarray(a_len, np.int32)
    b_len = np.ascontiguousarray(b_len, np.int32)
    npairs = a_len.shape[0]
    scores = np.empty(npairs, np.int32)
    counts = np.empty(npairs, np.uint64)
    sat = np.empty(npairs, np.uint8)
    if _lib().orc_count_batch(npairs, pp, _ptr(a_off, _i64p), _ptr(a_len, _i32p), _ptr(b_off, _i64p),
                              _ptr(b_len, _i32p), *scoring, _ptr(scores, _i32p), _ptr(counts, _u64p),
                              _ptr(sat, _u8p), int(nthreads)) < 0:
        raise MemoryError("oracle: out of host memory")
    return scores, counts, sat


def optimal_moves(H, a, b, i, j, scoring=PAPER_SCORING):
    """Moves into (i,j) whose candidate equals H(i,j), in the order D, U, L."""
    match, mismatch, gap = scoring
    if i == 0 and j == 0:
        return []
    if i == 0:
        return [L]
    if j == 0:
        return [U]
    h = int(H[i, j])
    out = []
    if int(H[i - 1, j - 1]) + (match if a[i - 1] == b[j - 1] else mismatch) == h:
        out.append(D)
    if int(H[i - 1, j]) + gap == h:
        out.append(U)
    if int(H[i, j - 1]) + gap == h:
        out.append(L)
    return out


def enumerate_paths(a, b, scoring=PAPER_SCORING, k: int = 1):
    """Up to k co-optimal paths (forward move strings), in depth-first order
    from (m,n) with moves tried D, then U, then L."""
    a = np.asarray(a, dtype=np.uint8)
    b = np.asarray(b, dtype=np.uint8)
    m, n = len(a), len(b)
    H = fill(a, b, scoring).astype(np.int64)
    out = []
    if k <= 0:
        return out
    # the search: the cell at each depth with its optimal moves and the next one to try
    cells = [(m, n)]
    opts = [optimal_moves(H, a, b, m, n, scoring)]
    nxt = [0]
    moves = []  # moves taken so far, from (m,n) backwards
    while cells and len(out) < k:
        i, j = cells[-1]
        if i == 0 and j == 0:
            out.append(np.array(moves[::-1], dtype=np.uint8))
        if nxt[-1] >= len(opts[-1]):
            cells.pop()
            opts.pop()
            nxt.pop()
            if moves:
                moves.pop()
            continue
        mv = opts[-1][nxt[-1]]
        nxt[-1] += 1
        ni, nj = (i - 1, j - 1) if mv == D else ((i - 1, j) if mv == U else (i, j - 1))
        moves.append(mv)
        cells.append((ni, nj))
        opts.append(optimal_moves(H, a, b, ni, nj, scoring))
        nxt.append(0)
    return out
