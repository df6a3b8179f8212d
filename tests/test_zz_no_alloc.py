"""nw_align_noalloc: nw_align on the library's fixed device scratch array,
for callers that cannot allocate.  Called through the C-ABI and compared
with nw_align (and the oracle) score for score and move for move, on two
calls in a row with the second smaller, on both single-pair engines (the
multi-wave one from 512 columns, the one-wave one below); a pair beyond the
scratch is rejected before any work; once the kernels have been dispatched
once, the calls leave the device's free memory unchanged."""
import ctypes

import numpy as np
import pytest

import oracle
from workloads import mutate, random_seq

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2412_21103_amd as nwp  # noqa: E402
from gpu_util import dev_u8, say  # noqa: E402

vp = ctypes.c_void_p


def _noalloc(da, db, score, path, plen, scoring=nwp.PAPER_SCORING, score_only=False):
    L = nwp.lib()
    m, n = da.numel(), db.numel()
    return L.nw_align_noalloc(vp(da.data_ptr()), m, vp(db.data_ptr()), n, nwp.Scoring(*scoring),
                              nwp.SCORE_ONLY if score_only else 0, vp(score.data_ptr()),
                              vp(path.data_ptr()) if path is not None else vp(0),
                              path.numel() if path is not None else 0,
                              vp(plen.data_ptr()) if plen is not None else vp(0),
                              vp(torch.cuda.current_stream().cuda_stream))


def _pair(rng, m, rate):
    a = random_seq(rng, m)
    return a, mutate(rng, a, rate)


@pytest.mark.parametrize("sizes", [(3000, 1200), (450, 200)], ids=["multi-wave", "one-wave"])
def test_noalloc_matches_nw_align_twice(sizes):
    assert nwp.lib().nw_init() == 0
    rng = np.random.default_rng(sizes[0])
    pairs = [_pair(rng, sizes[0], 0.1), _pair(rng, sizes[1], 0.2)]
    cap = max(len(a) + len(b) for a, b in pairs)
    # outputs allocated before the calls; the calls themselves allocate nothing
    ins = [(dev_u8(a), dev_u8(b)) for a, b in pairs]
    score = torch.empty(1, dtype=torch.int32, device="cuda")
    path = torch.empty(cap, dtype=torch.uint8, device="cuda")
    plen = torch.empty(1, dtype=torch.int64, device="cuda")
    score2 = torch.empty(1, dtype=torch.int32, device="cuda")
    # the runtime sets up each kernel at its first dispatch (code and private
    # memory), which can move the device's free memory once; warm up first
    for da, db in ins:
        assert _noalloc(da, db, score, path, plen) == 0
        assert _noalloc(da, db, score2, None, None, score_only=True) == 0
    torch.cuda.synchronize()
    for k, ((a, b), (da, db)) in enumerate(zip(pairs, ins)):
        say(f"noalloc: call {k}, {len(a)} x {len(b)}")
        free0 = torch.cuda.mem_get_info()[0]
        assert _noalloc(da, db, score, path, plen) == 0
        assert _noalloc(da, db, score2, None, None, score_only=True) == 0
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        s, p, pl = nwp.align(da, db)
        torch.cuda.synchronize()
        k_len = int(plen.item())
        assert int(score.item()) == int(s.item())
        assert int(score2.item()) == int(s.item())
        assert k_len == int(pl.item())
        assert torch.equal(path[:k_len], p[:k_len])
        s_ref, p_ref = oracle.align(a, b)
        assert int(score.item()) == s_ref
        assert path[:k_len].cpu().numpy().tolist() == p_ref.tolist()
    assert nwp.sync() is None


def test_noalloc_other_scoring_and_empty():
    rng = np.random.default_rng(5)
    score = torch.empty(1, dtype=torch.int32, device="cuda")
    path = torch.empty(4096, dtype=torch.uint8, device="cuda")
    plen = torch.empty(1, dtype=torch.int64, device="cuda")
    for m, n, sc in [(900, 700, (2, -3, -2)), (0, 17, (1, -1, -1)), (5, 0, (3, -1, -2))]:
        a = random_seq(rng, m)
        b = random_seq(rng, n)
        da, db = dev_u8(a), dev_u8(b)
        assert _noalloc(da, db, score, path, plen, sc) == 0
        torch.cuda.synchronize()
        s_ref, p_ref = oracle.align(a, b, sc)
        k = int(plen.item())
        assert int(score.item()) == s_ref
        assert path[:k].cpu().numpy().tolist() == p_ref.tolist()


def test_noalloc_rejects_beyond_scratch():
    assert nwp.align_noalloc_fits(8000, 8000)
    assert not nwp.align_noalloc_fits(20000, 20000)
    assert nwp.align_noalloc_fits(20000, 20000, score_only=True)
    # a pair too large for the scratch is refused before anything is queued
    # (the pointers are never read)
    L = nwp.lib()
    out = torch.empty(1, dtype=torch.int32, device="cuda")
    st = L.nw_align_noalloc(vp(out.data_ptr()), 20000, vp(out.data_ptr()), 20000, nwp.Scoring(1, -1, -1), 0,
                            vp(out.data_ptr()), vp(out.data_ptr()), 40000, vp(out.data_ptr()), vp(0))
    assert st == nwp.NW_ENOSPC
    # the usual argument checks come first
    st = L.nw_align_noalloc(vp(0), 10, vp(out.data_ptr()), 10, nwp.Scoring(1, -1, -1), 0,
                            vp(out.data_ptr()), vp(out.data_ptr()), 20, vp(out.data_ptr()), vp(0))
    assert st == nwp.NW_EINVAL
