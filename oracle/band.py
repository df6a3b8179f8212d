"""Band certificate and band labels (closed forms).

TEST INFRASTRUCTURE ONLY.

The paper's future-work paragraph (Sec. 5) asks for speed without missing an
optimal alignment; a band around the main diagonal is only safe if no optimal
path can leave it.  These closed forms decide that from a score alone.

Definitions, for a pair of lengths m (rows) and n (columns), Delta = n - m,
lo = min(0, Delta), hi = max(0, Delta):

* band(w) = cells (i, j) with lo - w <= j - i <= hi + w.
* A path that leaves band(w) reaches diagonal offset hi + w + 1 or lo - w - 1,
  so it has at least G = |Delta| + 2(w + 1) gap moves, and its number of
  diagonal moves is (m + n - G) / 2 <= min(m, n) - w - 1.  Its score is at most
  c_d * #D + gap * G with c_d = max(match, mismatch).  Written as a function
  of G this is c_d (m + n) / 2 + G (gap - c_d / 2), which falls with G when
  2 gap < c_d, so every such path scores at most

      U_out(w) = c_d * (min(m, n) - w - 1) + gap * (|Delta| + 2 w + 2).

* If w >= min(m, n) the band is the whole grid and nothing can leave it.
* A score S_R reached inside any region that contains band(w) certifies the
  region iff S_R > U_out(w) (strict): then every optimal path lies in the band,
  so the region-restricted fill has the same optimum and, because every cell
  on an optimal path keeps its exact value and its tied predecessors, the same
  tie-break path.  With equality an outside co-optimal path could win the tie
  break, so equality does not certify.
* w_cert(S) = smallest w >= 0 that certifies the true score S.
* w_path(path) = how far a path strays outside the corridor [lo, hi].
"""
from __future__ import annotations

import numpy as np

from . import D, U, L, PAPER_SCORING


def applicable(scoring=PAPER_SCORING) -> bool:
    match, mismatch, gap = scoring
    return 2 * gap < max(match, mismatch)


def u_out(m: int, n: int, w: int, scoring=PAPER_SCORING):
    """Upper bound on the score of any path that leaves band(w); None if no
    path can leave it."""
    match, mismatch, gap = scoring
    if w >= min(m, n):
        return None
    cd = max(match, mismatch)
    return cd * (min(m, n) - w - 1) + gap * (abs(n - m) + 2 * w + 2)


def certifies(s_region: int, m: int, n: int, w: int, scoring=PAPER_SCORING) -> bool:
    if not applicable(scoring):
        return False
    u = u_out(m, n, w, scoring)
    return True if u is None else s_region > u


def w_cert(s: int, m: int, n: int, scoring=PAPER_SCORING) -> int:
    """Smallest w >= 0 with s > U_out(w) (or min(m, n) if none smaller)."""
    match, mismatch, gap = scoring
    if not applicable(scoring):
        raise ValueError("certificate needs 2*gap < max(match, mismatch)")
    cd = max(match, mismatch)
    mn = min(m, n)
    # s > cd*(mn - w - 1) + gap*(|d| + 2w + 2)  <=>  w*(cd - 2 gap) > cd*(mn-1) + gap*(|d|+2) - s
    num = cd * (mn - 1) + gap * (abs(n - m) + 2) - s
    den = cd - 2 * gap
    w = num // den + 1 if num >= 0 else 0
    return int(max(0, min(w, mn)))


def in_band(i: int, j: int, m: int, n: int, w: int) -> bool:
    d = n - m
    return min(0, d) - w <= j - i <= max(0, d) + w


def w_path(path, m: int, n: int) -> int:
    """Largest excursion of a path outside the corridor [min(0,Delta), max(0,Delta)]."""
    d = n - m
    lo, hi = min(0, d), max(0, d)
    i = j = 0
    worst = 0
    for mv in np.asarray(path).tolist():
        if mv == D:
            i += 1
            j += 1
        elif mv == U:
            i += 1
        else:
            j += 1
        off = j - i
        worst = max(worst, off - hi, lo - off)
    return int(worst)


def band_cells(m: int, n: int, w: int) -> int:
    """Number of interior cells (1..m, 1..n) inside band(w)."""
    d = n - m
    lo, hi = min(0, d) - w, max(0, d) + w
    total = 0
    for i in range(1, m + 1):
        jl = max(1, i + lo)
        jh = min(n, i + hi)
        if jh >= jl:
            total += jh - jl + 1
    return total


__all__ = ["applicable", "u_out", "certifies", "w_cert", "in_band", "w_path", "band_cells"]


# ---------------------------------------------------------------------------
# A tighter certificate from the band's own scores.
#
# A path that leaves band(w) does so for the first time by a vertical move
# from the band's lowest diagonal (j - i = lo - w) or a horizontal move from
# its highest (j - i = hi + w): a diagonal move keeps j - i.  Up to the cell P
# it leaves from, the path stays in the band, so that part scores at most
# H_band(P), the best score of an in-band path from (0,0) to P.  The move
# adds gap, and the rest, from the first outside cell X = (i, j) to (m, n),
# has at most min(m-i, n-j) diagonal moves and at least |(m-i) - (n-j)| gaps:
#
#     suf(X) = gap * ((m-i) + (n-j)) + min(m-i, n-j) * max(c_d - 2 gap, 0)
#
# bounds it for every scoring.  So every leaving path scores at most
#
#     U_tight(w) = max over such moves P -> X of  H_band(P) + gap + suf(X),
#
# and a region score S > U_tight(w) certifies the band as before.  Each term
# is also bounded by U_out(w) (the closed form counts the same gaps), so the
# tight bound never certifies less.
# ---------------------------------------------------------------------------

NEG = None  # outside the band


def band_fill(a, b, w: int, scoring=PAPER_SCORING):
    """H_band over band(w) (None outside): the best score of a path from
    (0,0) that stays in band(w), by plain loops."""
    match, mismatch, gap = scoring
    m, n = len(a), len(b)
    H = [[NEG] * (n + 1) for _ in range(m + 1)]
    for i in range(m + 1):
        for j in range(n + 1):
            if not in_band(i, j, m, n, w):
                continue
            if i == 0 and j == 0:
                H[i][j] = 0
                continue
            best = None
            if i > 0 and j > 0 and H[i - 1][j - 1] is not None:
                best = H[i - 1][j - 1] + (match if a[i - 1] == b[j - 1] else mismatch)
            if i > 0 and H[i - 1][j] is not None:
                c = H[i - 1][j] + gap
                best = c if best is None else max(best, c)
            if j > 0 and H[i][j - 1] is not None:
                c = H[i][j - 1] + gap
                best = c if best is None else max(best, c)
            H[i][j] = best
    return H


def suffix_bound(i: int, j: int, m: int, n: int, scoring=PAPER_SCORING) -> int:
    match, mismatch, gap = scoring
    cd = max(match, mismatch)
    r, c = m - i, n - j
    return gap * (r + c) + min(r, c) * max(cd - 2 * gap, 0)


def u_tight(a, b, w: int, scoring=PAPER_SCORING):
    """``(S_band, U_tight)``: the best in-band score of (m,n) and the bound on
    every path that leaves band(w) (None if no path can leave it)."""
    gap = scoring[2]
    m, n = len(a), len(b)
    H = band_fill(a, b, w, scoring)
    d = n - m
    lo, hi = min(0, d) - w, max(0, d) + w
    best = None
    for i in range(m + 1):
        for j in range(n + 1):
            if H[i][j] is None:
                continue
            if j - i == lo and i + 1 <= m:      # vertical move out of the band
                t = H[i][j] + gap + suffix_bound(i + 1, j, m, n, scoring)
                best = t if best is None else max(best, t)
            if j - i == hi and j + 1 <= n:      # horizontal move out of the band
                t = H[i][j] + gap + suffix_bound(i, j + 1, m, n, scoring)
                best = t if best is None else max(best, t)
    return H[m][n], best


def certifies_tight(a, b, w: int, scoring=PAPER_SCORING) -> bool:
    s, u = u_tight(a, b, w, scoring)
    return True if u is None else s > u


def w_cert_tight(a, b, scoring=PAPER_SCORING) -> int:
    """Smallest w >= 0 that the tight bound certifies (min(m, n) at most:
    there no path can leave)."""
    m, n = len(a), len(b)
    for w in range(0, min(m, n) + 1):
        if certifies_tight(a, b, w, scoring):
            return w
    return min(m, n)
