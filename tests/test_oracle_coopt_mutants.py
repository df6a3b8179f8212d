"""The co-optimal count pins catch plausible mistakes: each case plants one
mistake in a copy of the oracle's C source (on the CPU), builds it, and
checks that a reduced pin suite (exhaustive enumeration, the Delannoy closed
form past 2^64) rejects it."""
import os
import subprocess
from math import comb

import numpy as np
import pytest

import oracle
from oracle import coopt
from pins import brute_force_all

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "nw_oracle.c")

MUTANTS = {
    "count_drops_vertical": ("            if (u == h) {\n                uint64_t t = s + N0[j];",
                             "            if (0) {\n                uint64_t t = s + N0[j];"),
    "left_reads_row_above": ("uint64_t t = s + N1[j - 1];", "uint64_t t = s + N0[j - 1];"),
    "first_column_zero": ("        N1[0] = 1;", "        N1[0] = 0;"),
    "flag_ignores_wrap": ("f |= (uint8_t)(F0[j] | (t < s));", "f |= (uint8_t)(F0[j]);"),
    "flag_not_inherited": ("f |= (uint8_t)(F1[j - 1] | (t < s));", "f |= (uint8_t)(t < s);"),
}


def _delannoy(m, n):
    return sum(comb(m, k) * comb(n, k) * 2 ** k for k in range(min(m, n) + 1))


def _pins_pass() -> bool:
    rng = np.random.default_rng(321)
    for _ in range(60):
        m, n = (int(x) for x in rng.integers(0, 6, 2))
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = rng.integers(0, 4, n).astype(np.uint8)
        for sc in [(1, -1, -1), (1, 0, 0)]:
            best, opt = brute_force_all(a, b, sc)
            if coopt.count(a, b, sc) != (best, len(opt), False):
                return False
    # (30, 24), (44, 18): the end cell's vertical addition is the first to
    # reach 2^64; (14, 73), (15, 63), (16, 55): only its horizontal
    # neighbour has reached it, and the sum does not wrap
    for m, n in [(20, 20), (30, 31), (40, 25), (30, 24), (44, 18), (14, 73), (15, 63), (16, 55)]:
        z = rng.integers(0, 4, m).astype(np.uint8), rng.integers(0, 4, n).astype(np.uint8)
        d = _delannoy(m, n)
        if coopt.count(*z, (-2, -2, -1)) != (-(m + n), d % (1 << 64), d >= (1 << 64)):
            return False
    return True


def test_unmodified_oracle_passes():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    c = tmp_path / "mut.c"
    so = tmp_path / "libmut.so"
    c.write_text(src.replace(old, new, 1))
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-fopenmp", str(c), "-o", str(so)], check=True)
    saved = oracle._lib, oracle._LIB_PATH, coopt._bound
    try:
        oracle._lib, oracle._LIB_PATH, coopt._bound = None, str(so), False
        assert not _pins_pass(), f"mutant {name} slipped through the pins"
    finally:
        oracle._lib, oracle._LIB_PATH, coopt._bound = saved
