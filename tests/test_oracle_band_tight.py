"""The band-edge bound (oracle/band.py ``u_tight``): pinned by enumeration,
and shown to reproduce the closed form exactly.

* every path that leaves band(w) scores at most u_tight (enumeration of all
  alignments, m, n <= 6, several scorings, including ones where the closed
  form does not apply);
* u_tight equals U_out(w) whenever some path can leave the band and the
  closed form applies: the all-gap exit from the first row (or column) with
  a suffix bounded by all matches is itself the closed form's worst case, so
  band-edge scores cannot tighten a certificate that knows nothing of the
  cells outside the band.
"""
import numpy as np
import pytest

from oracle import band
from pins import all_paths, path_score

SCORINGS = [(1, -1, -1), (2, -3, -2), (1, 0, -1), (-2, -2, -1), (1, -1, 0)]


def _leaving_max(a, b, w, sc):
    m, n = len(a), len(b)
    d = n - m
    lo, hi = min(0, d) - w, max(0, d) + w
    best = None
    for p in all_paths(m, n):
        i = j = 0
        out = False
        for mv in p:
            if mv == 1:
                i += 1
                j += 1
            elif mv == 2:
                i += 1
            else:
                j += 1
            out = out or not (lo <= j - i <= hi)
        if out:
            s = path_score(p, a, b, sc)
            best = s if best is None else max(best, s)
    return best


@pytest.mark.parametrize("sc", SCORINGS)
def test_bounds_every_leaving_path(sc):
    rng = np.random.default_rng(90)
    for _ in range(60):
        m, n = int(rng.integers(0, 7)), int(rng.integers(0, 7))
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = rng.integers(0, 4, n).astype(np.uint8)
        for w in range(0, 3):
            s_band, u = band.u_tight(a, b, w, sc)
            worst = _leaving_max(a, b, w, sc)
            assert (worst is None) == (u is None) or (worst is None and u is not None)
            if worst is not None:
                assert worst <= u, (a, b, w, sc)
            # the band's own score is the best in-band path to (m, n)
            assert s_band is not None


@pytest.mark.parametrize("sc", [s for s in SCORINGS if band.applicable(s)])
def test_equals_the_closed_form(sc):
    rng = np.random.default_rng(91)
    for _ in range(40):
        m, n = int(rng.integers(0, 40)), int(rng.integers(0, 40))
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = rng.integers(0, 4, n).astype(np.uint8)
        for w in (0, 1, 3, 7):
            _, u = band.u_tight(a, b, w, sc)
            assert u == band.u_out(m, n, w, sc), (m, n, w, sc)
