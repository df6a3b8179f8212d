"""CPU oracle for the Needleman-Wunsch hot path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may use this package; the product library never does.

* ``align``, ``score``, ``fill``, ``dirs``, ``align_batch``, ``allpairs`` wrap the
  plain C implementation in ``nw_oracle.c`` (paper Section 2, Eq. 1 read as the
  linear-gap recurrence; Section 3.2 and Eq. 2 for the all-pairs matrix).
* ``band`` holds the band certificate and its labels (closed forms).
* ``features`` and ``mlp`` hold the k-mer features and the band MLP reference.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None

PAPER_SCORING = (1, -1, -1)  # match, mismatch, gap (paper Sec. 2.3)
D, U, L = 1, 2, 3            # paper's direction codes (Sec. 3.1)

_u8p = ctypes.POINTER(ctypes.c_uint8)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L_ = ctypes.CDLL(_LIB_PATH)
        L_.orc_fill.argtypes = [_u8p, ctypes.c_int64, _u8p, ctypes.c_int64,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _i32p]
        L_.orc_fill.restype = None
        L_.orc_traceback.argtypes = [_i32p, _u8p, ctypes.c_int64, _u8p, ctypes.c_int64,
                                     ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _u8p]
        L_.orc_traceback.restype = ctypes.c_int64
        L_.orc_dirs.argtypes = [_i32p, _u8p, ctypes.c_int64, _u8p, ctypes.c_int64,
                                ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _u8p]
        L_.orc_dirs.restype = None
        L_.orc_score.argtypes = [_u8p, ctypes.c_int64, _u8p, ctypes.c_int64,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L_.orc_score.restype = ctypes.c_int32
        L_.orc_align.argtypes = [_u8p, ctypes.c_int64, _u8p, ctypes.c_int64,
                                 ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 _i32p, _u8p, _i64p, ctypes.c_int64]
        L_.orc_align.restype = ctypes.c_int
        L_.orc_align_batch.argtypes = [ctypes.c_int32, _u8p, _i64p, _i32p, _i64p, _i32p,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       _i32p, _u8p, _i64p, _i32p, ctypes.c_int32, ctypes.c_int64]
        L_.orc_align_batch.restype = ctypes.c_int64
        L_.orc_allpairs.argtypes = [ctypes.c_int32, _u8p, _i64p, _i32p,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    _i32p, ctypes.c_int32]
        L_.orc_allpairs.restype = None
        L_.orc_max_threads.argtypes = []
        L_.orc_max_threads.restype = ctypes.c_int
        _lib = L_
    return _lib


def _u8(x):
    x = np.ascontiguousarray(x, dtype=np.uint8)
    return x, x.ctypes.data_as(_u8p)


def _ptr(x, t):
    return x.ctypes.data_as(t)


def fill(a, b, scoring=PAPER_SCORING) -> np.ndarray:
    """Full (m+1) x (n+1) int32 score matrix."""
    a, pa = _u8(a)
    b, pb = _u8(b)
    m, n = a.shape[0], b.shape[0]
    H = np.empty((m + 1, n + 1), dtype=np.int32)
    lib().orc_fill(pa, m, pb, n, *scoring, _ptr(H, _i32p))
    return H


def traceback(H, a, b, scoring=PAPER_SCORING) -> np.ndarray:
    a, pa = _u8(a)
    b, pb = _u8(b)
    m, n = a.shape[0], b.shape[0]
    H = np.ascontiguousarray(H, dtype=np.int32)
    path = np.empty(m + n, dtype=np.uint8)
    k = lib().orc_traceback(_ptr(H, _i32p), pa, m, pb, n, *scoring, _ptr(path, _u8p))
    return path[:k].copy()


def dirs(a, b, scoring=PAPER_SCORING) -> np.ndarray:
    """Move code of every cell (0 at (0,0), 2 on column 0, 3 on row 0)."""
    H = fill(a, b, scoring)
    a, pa = _u8(a)
    b, pb = _u8(b)
    m, n = a.shape[0], b.shape[0]
    C = np.empty((m + 1, n + 1), dtype=np.uint8)
    lib().orc_dirs(_ptr(H, _i32p), pa, m, pb, n, *scoring, _ptr(C, _u8p))
    return C


def score(a, b, scoring=PAPER_SCORING) -> int:
    a, pa = _u8(a)
    b, pb = _u8(b)
    return int(lib().orc_score(pa, a.shape[0], pb, b.shape[0], *scoring))


def align(a, b, scoring=PAPER_SCORING, full_limit_bytes: int = 8 << 30):
    """Return ``(score, path)``; path holds moves 1/2/3 from (0,0) to (m,n)."""
    a, pa = _u8(a)
    b, pb = _u8(b)
    m, n = a.shape[0], b.shape[0]
    path = np.empty(max(m + n, 1), dtype=np.uint8)
    s = ctypes.c_int32(0)
    k = ctypes.c_int64(0)
    mode = lib().orc_align(pa, m, pb, n, *scoring, ctypes.byref(s), _ptr(path, _u8p),
                           ctypes.byref(k), int(full_limit_bytes))
    if mode < 0:
        raise MemoryError("oracle: out of host memory")
    return int(s.value), path[: k.value].copy()


def align_batch(pool, a_off, a_len, b_off, b_len, scoring=PAPER_SCORING, with_paths=True,
                nthreads: int = 0, full_limit_bytes: int = 1 << 30):
    """Batch of pairs from a pool.  Returns ``(scores, paths_list or None)``."""
    pool, pp = _u8(pool)
    a_off = np.ascontiguousarray(a_off, np.int64)
    b_off = np.ascontiguousarray(b_off, np.int64)
    a_len = np.ascontiguousarray(a_len, np.int32)
    b_len = np.ascontiguousarray(b_len, np.int32)
    npairs = a_len.shape[0]
    scores = np.empty(npairs, np.int32)
    if with_paths:
        caps = a_len.astype(np.int64) + b_len.astype(np.int64)
        path_off = np.concatenate([[0], np.cumsum(caps)[:-1]]).astype(np.int64) if npairs else np.zeros(0, np.int64)
        paths = np.empty(max(int(caps.sum()), 1), np.uint8)
        plen = np.empty(npairs, np.int32)
        r = lib().orc_align_batch(npairs, pp, _ptr(a_off, _i64p), _ptr(a_len, _i32p),
                                  _ptr(b_off, _i64p), _ptr(b_len, _i32p), *scoring,
                                  _ptr(scores, _i32p), _ptr(paths, _u8p), _ptr(path_off, _i64p),
                                  _ptr(plen, _i32p), int(nthreads), int(full_limit_bytes))
        if r < 0:
            raise MemoryError("oracle: out of host memory")
        out = [paths[path_off[k]: path_off[k] + plen[k]].copy() for k in range(npairs)]
        return scores, out
    r = lib().orc_align_batch(npairs, pp, _ptr(a_off, _i64p), _ptr(a_len, _i32p),
                              _ptr(b_off, _i64p), _ptr(b_len, _i32p), *scoring,
                              _ptr(scores, _i32p), None, None, None, int(nthreads),
                              int(full_limit_bytes))
    return scores, None


def allpairs(pool, off, lens, scoring=PAPER_SCORING, nthreads: int = 0) -> np.ndarray:
    pool, pp = _u8(pool)
    off = np.ascontiguousarray(off, np.int64)
    lens = np.ascontiguousarray(lens, np.int32)
    nseq = lens.shape[0]
    out = np.empty((nseq, nseq), np.int32)
    lib().orc_allpairs(nseq, pp, _ptr(off, _i64p), _ptr(lens, _i32p), *scoring,
                       _ptr(out, _i32p), int(nthreads))
    return out


def max_threads() -> int:
    return int(lib().orc_max_threads())


def rescore(path, a, b, scoring=PAPER_SCORING):
    """Score of an explicit move string, and whether it consumes a and b exactly."""
    match, mismatch, gap = scoring
    i = j = 0
    s = 0
    m, n = len(a), len(b)
    for mv in np.asarray(path).tolist():
        if mv == D:
            if i >= m or j >= n:
                return None, False
            s += match if a[i] == b[j] else mismatch
            i += 1
            j += 1
        elif mv == U:
            if i >= m:
                return None, False
            s += gap
            i += 1
        elif mv == L:
            if j >= n:
                return None, False
            s += gap
            j += 1
        else:
            return None, False
    return s, (i == m and j == n)
