"""Independent formulations that pin the oracle (no shared code with it).

* ``brute_force``: enumerate every alignment (every monotone path of diagonal,
  vertical and horizontal moves from (0,0) to (m,n)), score each one directly
  from its definition, and pick the optimum whose reversed move string is
  largest under D > U > L.  Greedy backtracking that prefers D, then U, then L
  at each cell yields exactly that path: at every step it takes the largest
  move that still lies on some optimal path.
* ``weighted_edit_distance``: textbook Wagner-Fischer minimum-cost edit
  distance.  For an alignment with M matches, X mismatches and G gaps,
  m + n = 2M + 2X + G, so
      2 S = match*(m+n) - [2 (match - mismatch) X + (match - 2 gap) G],
  i.e. maximising S is minimising an edit cost with substitution
  2 (match - mismatch) and indel (match - 2 gap).
"""
from __future__ import annotations

import numpy as np

D, U, L = 1, 2, 3
_RANK = {D: 2, U: 1, L: 0}


def all_paths(m: int, n: int):
    """Yield every move tuple from (0,0) to (m,n)."""
    out = []

    def rec(i, j, acc):
        if i == m and j == n:
            out.append(tuple(acc))
            return
        if i < m and j < n:
            acc.append(D)
            rec(i + 1, j + 1, acc)
            acc.pop()
        if i < m:
            acc.append(U)
            rec(i + 1, j, acc)
            acc.pop()
        if j < n:
            acc.append(L)
            rec(i, j + 1, acc)
            acc.pop()

    rec(0, 0, [])
    return out


def path_score(path, a, b, scoring):
    match, mismatch, gap = scoring
    i = j = 0
    s = 0
    for mv in path:
        if mv == D:
            s += match if a[i] == b[j] else mismatch
            i += 1
            j += 1
        elif mv == U:
            s += gap
            i += 1
        else:
            s += gap
            j += 1
    return s


def brute_force(a, b, scoring=(1, -1, -1)):
    """(best score, tie-break path) by exhaustive enumeration."""
    a = list(a)
    b = list(b)
    best = None
    best_key = None
    best_path = None
    for p in all_paths(len(a), len(b)):
        s = path_score(p, a, b, scoring)
        key = tuple(_RANK[x] for x in reversed(p))
        if best is None or s > best or (s == best and key > best_key):
            best, best_key, best_path = s, key, p
    return best, np.asarray(best_path, dtype=np.uint8)


def max_score_leaving_band(a, b, w, scoring=(1, -1, -1)):
    """Best score over paths that leave band(w); None if none leaves."""
    m, n = len(a), len(b)
    d = n - m
    lo, hi = min(0, d) - w, max(0, d) + w
    best = None
    for p in all_paths(m, n):
        i = j = 0
        out = False
        for mv in p:
            if mv == D:
                i += 1
                j += 1
            elif mv == U:
                i += 1
            else:
                j += 1
            if not (lo <= j - i <= hi):
                out = True
                break
        if out:
            s = path_score(p, a, b, scoring)
            best = s if best is None else max(best, s)
    return best


def weighted_edit_distance(a, b, sub_cost, indel_cost):
    m, n = len(a), len(b)
    prev = [j * indel_cost for j in range(n + 1)]
    for i in range(1, m + 1):
        cur = [i * indel_cost] + [0] * n
        ai = a[i - 1]
        for j in range(1, n + 1):
            c_sub = prev[j - 1] + (0 if ai == b[j - 1] else sub_cost)
            c_del = prev[j] + indel_cost
            c_ins = cur[j - 1] + indel_cost
            cur[j] = min(c_sub, c_del, c_ins)
        prev = cur
    return prev[n]


def score_from_edit_distance(a, b, scoring):
    match, mismatch, gap = scoring
    dist = weighted_edit_distance(list(a), list(b), 2 * (match - mismatch), match - 2 * gap)
    total = match * (len(a) + len(b)) - dist
    assert total % 2 == 0
    return total // 2


def brute_force_all(a, b, scoring=(1, -1, -1)):
    """Every optimal alignment, by exhaustive enumeration, in decreasing order
    of the reversed move string under D > U > L."""
    a = list(a)
    b = list(b)
    scored = [(path_score(p, a, b, scoring), p) for p in all_paths(len(a), len(b))]
    best = max(s for s, _ in scored)
    opt = [p for s, p in scored if s == best]
    opt.sort(key=lambda p: tuple(_RANK[x] for x in reversed(p)), reverse=True)
    return best, opt
