"""Bit-exact parity of the HIP path against the CPU oracle (scores and paths)."""
import numpy as np
import pytest

import oracle
from workloads import (config_allpairs, config_batch, config_single, mutate, pack_pairs,
                       pack_seqs, random_seq)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import gpu_align, gpu_allpairs, gpu_batch, say  # noqa: E402

P = (1, -1, -1)
EDGE = [0, 1, 2, 15, 16, 17, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1023, 1024,
        1025]


def check_pair(a, b, sc=P, tag=""):
    s_ref, p_ref = oracle.align(a, b, sc)
    s, p = gpu_align(a, b, sc)
    assert s == s_ref, (tag, len(a), len(b), s, s_ref)
    assert p.tolist() == p_ref.tolist(), (tag, len(a), len(b))
    s2, _ = gpu_align(a, b, sc, score_only=True)
    assert s2 == s_ref, (tag, "score-only", len(a), len(b))


def test_single_pair_config_1024():
    p = config_single()
    say("single 1024x1024")
    check_pair(p.a[0], p.b[0], P, "config_single")


def test_single_pair_edge_shapes():
    rng = np.random.default_rng(21)
    for m in EDGE:
        for n in [0, 1, 17, 64, 65, 300, 513, 1025]:
            say(f"edge m={m} n={n}")
            a = random_seq(rng, m)
            b = mutate(rng, a, 0.1)[:n] if n <= m else random_seq(rng, n)
            check_pair(a, b, P, "edge")


def test_single_pair_identical_and_related():
    rng = np.random.default_rng(22)
    for L in [1, 100, 777, 1500]:
        a = random_seq(rng, L)
        say(f"identical L={L}")
        s, p = gpu_align(a, a.copy())
        assert s == L and p.tolist() == [1] * L
        b = mutate(rng, a, 0.15)
        check_pair(a, b, P, "related")


@pytest.mark.parametrize("sc", [(2, -3, -2), (1, 0, -1), (3, -1, -2), (5, -4, -3), (1, -1, -2)])
def test_other_scorings(sc):
    rng = np.random.default_rng(23)
    for m, n in [(50, 61), (300, 280), (700, 720)]:
        a = random_seq(rng, m)
        b = mutate(rng, a, 0.2)[:n]
        say(f"scoring {sc} m={m} n={len(b)}")
        check_pair(a, b, sc, "scoring")


def test_batch_matches_oracle():
    pairs = config_batch(seed=31, npairs=300, lo=1, hi=700)
    pool, ao, al, bo, bl = pack_pairs(pairs)
    max_len = int(max(al.max(), bl.max()))
    say(f"batch 300 pairs max_len={max_len}")
    s_ref, p_ref = oracle.align_batch(pool, ao, al, bo, bl, P)
    s, paths, plen = gpu_batch(pool, ao, al, bo, bl, max_len, P)
    assert (s == s_ref).all(), np.nonzero(s != s_ref)
    for k in range(len(pairs)):
        assert paths[k].tolist() == p_ref[k].tolist(), k
    s2, _ = gpu_batch(pool, ao, al, bo, bl, max_len, P, score_only=True)
    assert (s2 == s_ref).all()


def test_batch_with_smaller_workspace():
    # a workspace below the full-occupancy size runs fewer waves, same results;
    # one below a single block of slots is rejected before any launch
    import paper_2412_21103_amd as nwp
    pairs = config_batch(seed=33, npairs=200, lo=1, hi=900)
    pool, ao, al, bo, bl = pack_pairs(pairs)
    max_len = int(max(al.max(), bl.max()))
    full = nwp.batch_workspace_size(len(pairs), max_len)
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")
    args = [t(pool, np.uint8), t(ao, np.int64), t(al, np.int32), t(bo, np.int64), t(bl, np.int32)]
    s_ref, p_ref = oracle.align_batch(pool, ao, al, bo, bl, P)
    for frac in (4, 37):
        say(f"batch workspace 1/{frac}")
        ws = torch.empty(full // frac, dtype=torch.uint8, device="cuda")
        s, paths, poff, plen = nwp.align_batch(*args, max_len, P, workspace=ws)
        torch.cuda.synchronize()
        s, paths, poff, plen = (x.cpu().numpy() for x in (s, paths, poff, plen))
        assert (s == s_ref).all()
        for k in range(len(pairs)):
            assert paths[poff[k]:poff[k] + plen[k]].tolist() == p_ref[k].tolist(), (frac, k)
    tiny = torch.empty(4096, dtype=torch.uint8, device="cuda")
    out = torch.empty(len(pairs), dtype=torch.int32, device="cuda")
    st = nwp.lib().nw_align_batch(len(pairs), nwp._ptr(args[0]), nwp._ptr(args[1]), nwp._ptr(args[2]),
                                  nwp._ptr(args[3]), nwp._ptr(args[4]), max_len, nwp.Scoring(*P),
                                  nwp.SCORE_ONLY, nwp._ptr(out), None, None, None, nwp._ptr(tiny),
                                  tiny.numel(), None)
    assert st == nwp.NW_ENOSPC


def test_batch_pair_beyond_max_len_is_flagged():
    rng = np.random.default_rng(32)
    A = [random_seq(rng, 50), random_seq(rng, 120), random_seq(rng, 30)]
    B = [random_seq(rng, 40), random_seq(rng, 60), random_seq(rng, 30)]
    pool, off, lens = pack_seqs([x for ab in zip(A, B) for x in ab])
    ao, bo, al, bl = off[0::2], off[1::2], lens[0::2], lens[1::2]
    say("batch with an over-long pair")
    s, paths, plen = gpu_batch(pool, ao, al, bo, bl, 100, P)
    assert s[1] == np.iinfo(np.int32).min and plen[1] == -1
    for k in (0, 2):
        s_ref, p_ref = oracle.align(A[k], B[k], P)
        assert s[k] == s_ref and paths[k].tolist() == p_ref.tolist()


def test_allpairs_matches_oracle():
    seqs = config_allpairs(seed=41, nseq=40, lo=20, hi=600, root_len=1000)
    pool, off, lens = pack_seqs(seqs)
    say("allpairs 40 sequences")
    M_ref = oracle.allpairs(pool, off, lens, P)
    M = gpu_allpairs(pool, off, lens, int(lens.max()), P)
    assert (M == M_ref).all()
    assert (M == M.T).all() and (np.diag(M) == lens).all()


@pytest.fixture
def walk_limit(request):
    import paper_2412_21103_amd as nwp
    nwp.set_walk_limit(request.param)
    yield request.param
    nwp.set_walk_limit(0)


@pytest.mark.parametrize("walk_limit", [1 << 30, 1], indirect=True, ids=["one_wave_walk", "strip_parallel_walk"])
def test_cooperative_single_pair_shapes(walk_limit):
    # one pair with n >= 512 runs on many waves; cover tiny m, strip-multiple
    # and ragged n, and long m; every path traced back by one wave, and every
    # path by the strip-parallel walk
    rng = np.random.default_rng(24)
    for m, n in [(1, 512), (2, 4096), (17, 640), (100, 5000), (3000, 2999), (4097, 4096),
                 (700, 8193), (9000, 1100)]:
        a = random_seq(rng, m)
        b = mutate(rng, random_seq(rng, n), 0.0) if m < 50 else mutate(rng, a, 0.12)[:n]
        if len(b) < n:
            b = np.concatenate([b, random_seq(rng, n - len(b))])
        say(f"coop m={m} n={n} walk limit {walk_limit}")
        check_pair(a, b, P, "coop")


@pytest.mark.parametrize("walk_limit", [1], indirect=True)
def test_cooperative_traceback_both_chains(walk_limit):
    # The strip-parallel traceback places every strip's segment at once when each
    # re-walk from a strip's true entry meets that strip's speculative walk,
    # and falls back to chaining the strips one by one when one does not.
    # Periodic and unrelated sequences have parallel co-optimal paths that
    # never meet inside a strip, so they take the fallback; a related pair
    # takes the parallel placement.  The chain taken is read from the
    # workspace (its header: a fallback flag at int32 index 32 + 4).
    import torch
    import paper_2412_21103_amd as nwp
    rng = np.random.default_rng(77)
    unit = random_seq(rng, 20)
    a_rep = np.tile(unit, 160)[:3000]
    b_rep = np.concatenate([random_seq(rng, 11), mutate(rng, a_rep, 0.05)])[:3003]
    a_rel = random_seq(rng, 3000)
    b_rel = mutate(rng, a_rel, 0.3)
    cases = [("periodic", a_rep, b_rep, 1), ("unrelated", random_seq(rng, 3000), random_seq(rng, 2900), 1),
             ("related", a_rel, b_rel, None)]
    for tag, a, b, want in cases:
        m, n = len(a), len(b)
        ws = torch.zeros(nwp.align_workspace_size(m, n), dtype=torch.uint8, device="cuda")
        s, p, pl = nwp.align(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), P, workspace=ws)
        torch.cuda.synchronize()
        fallback = int(ws[128 + 16:128 + 20].cpu().numpy().view(np.int32)[0])
        say(f"traceback chain {tag} {m}x{n}: fallback={fallback}")
        s_ref, p_ref = oracle.align(a, b, P)
        k = int(pl.item())
        assert int(s.item()) == s_ref, tag
        assert p[:k].cpu().numpy().tolist() == p_ref.tolist(), tag
        if want is not None:
            assert fallback == want, tag


def test_long_pair_full_size():
    from workloads import config_long_pair
    p = config_long_pair()
    a, b = p.a[0], p.b[0]
    say(f"long pair {len(a)} x {len(b)}: GPU")
    s, path = gpu_align(a, b)
    say("long pair: oracle (two-row mode)")
    s_ref, p_ref = oracle.align(a, b, P, full_limit_bytes=0)
    assert s == s_ref
    assert path.tolist() == p_ref.tolist()
    r, ok = oracle.rescore(path, a, b, P)
    assert ok and r == s
