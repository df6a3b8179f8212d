"""The pins catch plausible mistakes: each case below plants one mistake in a
copy of the oracle's C source (on the CPU), builds it, and checks that the pin
suite rejects it."""
import json
import os
import subprocess

import numpy as np
import pytest

import oracle
from pins import brute_force, score_from_edit_distance

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "nw_oracle.c")

MUTANTS = {
    "left_gap_sign": ("int32_t l = row[j - 1] + gap;", "int32_t l = row[j - 1] - gap;"),
    "boundary_row_sign": ("for (int64_t j = 1; j <= n; ++j) H[j] = (int32_t)(j * gap);",
                          "for (int64_t j = 1; j <= n; ++j) H[j] = (int32_t)(-j * gap);"),
    "match_mismatch_swapped": ("return x == y ? match : mismatch;", "return x == y ? mismatch : match;"),
    "diag_reads_up": ("int32_t d = up[j - 1] + subst(a[i - 1], b[j - 1], match, mismatch);",
                      "int32_t d = up[j] + subst(a[i - 1], b[j - 1], match, mismatch);"),
    "dropped_left_term": ("    if (l > r) r = l;\n", "\n"),
    "tie_prefers_up": ("        if (h == d) return ORC_D;",
                       "        if (h == d && !(h == H[(i - 1) * W + j] + gap)) return ORC_D;"),
    "traceback_diag_keeps_column": ("        if (mv == ORC_D) { --i; --j; }\n        else if (mv == ORC_U) { --i; }\n        else { --j; }\n    }\n    for (int64_t p = 0, q = k - 1; p < q; ++p, --q) {\n        uint8_t t = path[p]; path[p] = path[q]; path[q] = t;\n    }\n    return k;",
                                    "        if (mv == ORC_D) { --i; }\n        else if (mv == ORC_U) { --i; }\n        else { --j; }\n    }\n    for (int64_t p = 0, q = k - 1; p < q; ++p, --q) {\n        uint8_t t = path[p]; path[p] = path[q]; path[q] = t;\n    }\n    return k;"),
    "path_not_reversed": ("    for (int64_t p = 0, q = k - 1; p < q; ++p, --q) {\n        uint8_t t = path[p]; path[p] = path[q]; path[q] = t;\n    }\n    return k;",
                          "    return k;"),
}


def _pins_pass() -> bool:
    """A reduced pin suite; returns False at the first failure."""
    rng = np.random.default_rng(123)
    for case in json.load(open(os.path.join(HERE, "golden", "hand_examples.json")))["cases"]:
        code = {"A": 0, "C": 1, "G": 2, "T": 3}
        a = np.array([code[c] for c in case["a"]], np.uint8)
        b = np.array([code[c] for c in case["b"]], np.uint8)
        s, p = oracle.align(a, b, tuple(case["scoring"]))
        if s != case["score"] or p.tolist() != case["path"]:
            return False
    for _ in range(40):
        m, n = rng.integers(0, 6, 2)
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = rng.integers(0, 4, n).astype(np.uint8)
        s_bf, p_bf = brute_force(a, b)
        s, p = oracle.align(a, b)
        if s != s_bf or p.tolist() != p_bf.tolist():
            return False
    for _ in range(10):
        m, n = rng.integers(0, 50, 2)
        a = rng.integers(0, 4, m).astype(np.uint8)
        b = rng.integers(0, 4, n).astype(np.uint8)
        if oracle.score(a, b) != score_from_edit_distance(a, b, (1, -1, -1)):
            return False
    return True


def test_unmodified_oracle_passes():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    c = tmp_path / "mut.c"
    so = tmp_path / "libmut.so"
    c.write_text(mutated)
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-fopenmp", str(c), "-o", str(so)],
                   check=True)
    saved_lib, saved_path = oracle._lib, oracle._LIB_PATH
    try:
        oracle._lib = None
        oracle._LIB_PATH = str(so)
        assert not _pins_pass(), f"mutant {name} slipped through the pins"
    finally:
        oracle._lib, oracle._LIB_PATH = saved_lib, saved_path
    # sanity: the real oracle is back
    assert oracle.score(np.zeros(3, np.uint8), np.zeros(3, np.uint8)) == 3
