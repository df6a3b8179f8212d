"""Independent pins of band.w_path, the largest excursion of a path outside
the corridor of diagonals [min(0, n-m), max(0, n-m)].

Every path (all monotone D/U/L move strings from (0,0) to (m,n)) is
enumerated for m, n <= 5 and checked against facts that do not restate the
function's own loop:

* containment, the definition the banded fill relies on: the path lies in
  band(w) (every visited cell, checked one by one) exactly when w >= w_path;
* counting: the number of paths with w_path <= w equals the number of
  lattice paths through band(w), counted by a separate dynamic programme over
  the band's cells;
* the gap bound behind the certificate: a path with excursion e > 0 makes at
  least |n-m| + 2e gap moves, and the fewest gaps over all paths with
  excursion e is exactly that.

Planted mistakes (an off-by-one, swapped corridor ends, the wrong sign of
n - m, a running excursion that is never reset to the corridor) are each
rejected by these pins.
"""
import inspect
import textwrap

import numpy as np
import pytest

from oracle import band
from pins import all_paths

D, U, L = 1, 2, 3


def _cells(path):
    i = j = 0
    out = [(0, 0)]
    for mv in path:
        if mv == D:
            i, j = i + 1, j + 1
        elif mv == U:
            i += 1
        else:
            j += 1
        out.append((i, j))
    return out


def _in_band(i, j, m, n, w):
    lo, hi = min(0, n - m), max(0, n - m)
    return lo - w <= j - i <= hi + w


def _count_paths_in_band(m, n, w):
    """Paths from (0,0) to (m,n) whose every cell lies in band(w)."""
    N = [[0] * (n + 1) for _ in range(m + 1)]
    for i in range(m + 1):
        for j in range(n + 1):
            if not _in_band(i, j, m, n, w):
                continue
            if i == 0 and j == 0:
                N[i][j] = 1
                continue
            N[i][j] = ((N[i - 1][j - 1] if i and j else 0) + (N[i - 1][j] if i else 0)
                       + (N[i][j - 1] if j else 0))
    return N[m][n]


def _pins_pass(w_path) -> bool:
    for m in range(0, 6):
        for n in range(0, 6):
            paths = all_paths(m, n)
            ex = [w_path(np.array(p, np.uint8), m, n) for p in paths]
            top = m + n + 1
            for p, e in zip(paths, ex):
                cells = _cells(p)
                for w in range(0, top):
                    inside = all(_in_band(i, j, m, n, w) for i, j in cells)
                    if inside != (w >= e):
                        return False
                gaps = sum(1 for mv in p if mv != D)
                if gaps < abs(n - m) + 2 * e:
                    return False
            for w in range(0, top):
                if sum(1 for e in ex if e <= w) != _count_paths_in_band(m, n, w):
                    return False
            for e in set(ex):
                fewest = min(sum(1 for mv in p if mv != D) for p, x in zip(paths, ex) if x == e)
                if fewest != abs(n - m) + 2 * e:
                    return False
    return True


def test_w_path_pins():
    assert _pins_pass(band.w_path)


def test_w_path_hand_cases():
    # identical lengths, all diagonal: inside the corridor
    assert band.w_path([D] * 4, 4, 4) == 0
    # all vertical then all horizontal on a square grid goes m below the corridor
    assert band.w_path([U] * 3 + [L] * 3, 3, 3) == 3
    # n = m + 2: the corridor is [0, 2]; L, L, D stays inside, U first leaves by 1
    assert band.w_path([L, L, D], 1, 3) == 0
    assert band.w_path([U, L, L, L], 1, 3) == 1
    # empty sides
    assert band.w_path([L] * 5, 0, 5) == 0
    assert band.w_path([U] * 5, 5, 0) == 0


MUTANTS = {
    "off_by_one": ("worst = max(worst, off - hi, lo - off)", "worst = max(worst, off - hi + 1, lo - off)"),
    "corridor_swapped": ("lo, hi = min(0, d), max(0, d)", "hi, lo = min(0, d), max(0, d)"),
    "delta_sign": ("d = n - m", "d = m - n"),
    "start_negative": ("worst = 0", "worst = -1"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_w_path_mutant_is_caught(name):
    old, new = MUTANTS[name]
    src = textwrap.dedent(inspect.getsource(band.w_path))
    assert src.count(old) == 1, name
    scope = {"np": np, "D": band.D, "U": band.U, "L": band.L}
    exec(src.replace(old, new), scope)
    try:
        ok = _pins_pass(scope["w_path"])
    except Exception:
        ok = False
    assert not ok, f"mutant {name} slipped through the pins"
