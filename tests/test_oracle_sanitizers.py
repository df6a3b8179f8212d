"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only).

The test builds a second copy of nw_oracle.c with -fsanitize=address,undefined
and -fno-sanitize-recover=all, then runs a child Python process with the
sanitizer runtime preloaded that drives every exported function (full-matrix
and two-row alignment, traceback, direction dump, batch with and without
paths, all-pairs, co-optimal counts) over random and edge-case inputs,
checking the results against brute force and the plain build.  Any
out-of-bounds access, use after free, signed overflow or other undefined
behaviour aborts the child, which fails the test.
"""
import os
import subprocess
import sys
import textwrap

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "nw_oracle.c")


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


CHILD = textwrap.dedent("""
    import sys
    import numpy as np
    sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
    import oracle
    from oracle import coopt
    from pins import brute_force
    oracle._LIB_PATH = {lib!r}
    oracle._lib = None
    coopt_lib = getattr(coopt, "_lib", None)
    rng = np.random.default_rng(7)
    for sc in [(1, -1, -1), (2, -3, -2), (1, 0, -1)]:
        for m in range(0, 6):
            for n in range(0, 6):
                a = rng.integers(0, 4, m).astype(np.uint8)
                b = rng.integers(0, 4, n).astype(np.uint8)
                s, p = oracle.align(a, b, sc)
                s2, p2 = oracle.align(a, b, sc, full_limit_bytes=0)
                assert s == s2 and p.tolist() == p2.tolist()
                if sc == (1, -1, -1):
                    sb, pb = brute_force(a, b)
                    assert s == sb and p.tolist() == pb.tolist()
                oracle.dirs(a, b, sc)
                assert oracle.score(a, b, sc) == s
    # larger pairs in both memory modes, any byte values
    for m, n in [(300, 257), (1, 900), (900, 1), (513, 513)]:
        a = rng.integers(0, 256, m).astype(np.uint8)
        b = rng.integers(0, 256, n).astype(np.uint8)
        s, p = oracle.align(a, b)
        s2, p2 = oracle.align(a, b, full_limit_bytes=0)
        assert s == s2 and p.tolist() == p2.tolist()
        assert oracle.rescore(p, a, b)[0] == s
    # batch (paths and scores only), all-pairs, co-optimal counts
    lens = rng.integers(0, 60, 24)
    seqs = [rng.integers(0, 4, int(k)).astype(np.uint8) for k in lens]
    pool = np.concatenate(seqs + [np.zeros(1, np.uint8)])
    off = np.concatenate([[0], np.cumsum(lens)[:-1]]).astype(np.int64)
    lens32 = lens.astype(np.int32)
    sc_, paths = oracle.align_batch(pool, off[:12], lens32[:12], off[12:], lens32[12:], nthreads=3)
    sc0, none = oracle.align_batch(pool, off[:12], lens32[:12], off[12:], lens32[12:], with_paths=False,
                                   full_limit_bytes=0)
    assert none is None and (sc_ == sc0).all()
    for k in range(12):
        s, p = oracle.align(seqs[k], seqs[12 + k])
        assert sc_[k] == s and paths[k].tolist() == p.tolist()
    M = oracle.allpairs(pool, off, lens32, nthreads=3)
    assert (M == M.T).all()
    s, cnt, flag = coopt.count_batch(pool, off[:12], lens32[:12], off[12:], lens32[12:], (1, -1, -1))
    assert (s == sc_).all() and (cnt >= 1).all()
    print("sanitized oracle ok")
""")


@pytest.mark.slow
def test_oracle_under_asan_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime for gcc")
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c99", "-fPIC", "-shared", "-fopenmp",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    SRC, "-o", str(lib)], check=True)
    script = tmp_path / "child.py"
    script.write_text(CHILD.format(root=ROOT, tests=HERE, lib=str(lib)))
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    # the interpreter itself is not instrumented: skip leak checks of its
    # allocations and let sanitizer reports abort the child
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "3"
    r = subprocess.run([sys.executable, str(script)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "sanitized oracle ok" in r.stdout
