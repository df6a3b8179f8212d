"""Argument checks and reduced workspaces of nw_cooptimal and nw_center_star,
through the C-ABI: errors are reported before any work is queued, and a
workspace with fewer wave slots gives the same results as the full one."""
import ctypes

import numpy as np
import pytest

from oracle import coopt
from workloads import Pairs, mutate, pack_pairs, pack_seqs, random_seq

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2412_21103_amd as nwp  # noqa: E402

P = nwp.Scoring(1, -1, -1)
vp = ctypes.c_void_p


def ptr(x):
    return vp(x.data_ptr()) if x is not None else vp(0)


def _dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")


def _pairs(seed, npairs, lo, hi):
    rng = np.random.default_rng(seed)
    a = [random_seq(rng, int(rng.integers(lo, hi))) for _ in range(npairs)]
    pr = Pairs(a, [mutate(rng, x, 0.15) for x in a], "errors")
    pool, ao, al, bo, bl = pack_pairs(pr)
    ml = int(max(al.max(), bl.max()))
    return (pool, ao, al, bo, bl), [_dev(pool, np.uint8), _dev(ao, np.int64), _dev(al, np.int32),
                                    _dev(bo, np.int64), _dev(bl, np.int32)], ml


def _co(L, npairs, d, ml, k, ws, nbytes, outs):
    scores, counts, sat, paths, poff, plen, npaths = outs
    return L.nw_cooptimal(npairs, *[ptr(x) for x in d], ml, P, ptr(scores), ptr(counts), ptr(sat), k, ptr(paths),
                          ptr(poff), ptr(plen), ptr(npaths), ptr(ws), nbytes, vp(torch.cuda.current_stream().cuda_stream))


def _outs(npairs, al, bl, k):
    dev = "cuda"
    caps = (al.astype(np.int64) + bl.astype(np.int64)) * max(k, 1)
    poff = _dev(np.concatenate([[0], np.cumsum(caps)[:-1]]), np.int64)
    return (torch.empty(npairs, dtype=torch.int32, device=dev), torch.empty(npairs, dtype=torch.int64, device=dev),
            torch.empty(npairs, dtype=torch.uint8, device=dev),
            torch.empty(int(caps.sum()), dtype=torch.uint8, device=dev), poff,
            torch.zeros((npairs, max(k, 1)), dtype=torch.int32, device=dev),
            torch.empty(npairs, dtype=torch.int32, device=dev))


def test_cooptimal_argument_errors():
    L = nwp.lib()
    packed, d, ml = _pairs(60, 8, 50, 90)
    outs = _outs(8, packed[2], packed[4], 2)
    full = nwp.cooptimal_workspace_size(8, ml, 2)
    ws = torch.empty(full, dtype=torch.uint8, device="cuda")
    assert _co(L, 8, d, ml, -1, ws, full, outs) == nwp.NW_EINVAL
    assert _co(L, -1, d, ml, 0, ws, full, outs) == nwp.NW_EINVAL
    assert _co(L, 8, [d[0], None, d[2], d[3], d[4]], ml, 0, ws, full, outs) == nwp.NW_EINVAL
    # k > 0 needs the path arrays
    assert _co(L, 8, d, ml, 2, ws, full, (outs[0], outs[1], outs[2], None, None, None, None)) == nwp.NW_EINVAL
    assert _co(L, 8, d, ml, 2, ws, 1024, outs) == nwp.NW_ENOSPC
    assert _co(L, 1 << 20, d, ml, 1 << 12, ws, full, outs) == nwp.NW_ERANGE
    assert _co(L, 0, d, ml, 0, None, 0, outs) == nwp.NW_OK
    torch.cuda.synchronize()


@pytest.mark.parametrize("k,lo,hi", [(0, 20, 400), (3, 20, 400), (0, 200, 1300)])
def test_cooptimal_smaller_workspace_same_results(k, lo, hi):
    """With k = 0 pairs of 2^16 cells or more are filled by the four waves of
    a block; a smaller workspace runs fewer blocks and waves."""
    L = nwp.lib()
    npairs = 300
    packed, d, ml = _pairs(61, npairs, lo, hi)
    full = nwp.cooptimal_workspace_size(npairs, ml, k)
    ws = torch.empty(full, dtype=torch.uint8, device="cuda")
    a = _outs(npairs, packed[2], packed[4], k)
    assert _co(L, npairs, d, ml, k, ws, full, a) == nwp.NW_OK
    b = _outs(npairs, packed[2], packed[4], k)
    assert _co(L, npairs, d, ml, k, ws, full // 9, b) == nwp.NW_OK
    torch.cuda.synchronize()
    for x, y in zip(a[:3], b[:3]):
        assert torch.equal(x, y)
    if k:
        assert torch.equal(a[6], b[6]) and torch.equal(a[5], b[5])
        pa, pb, poff, plen = a[3].cpu().numpy(), b[3].cpu().numpy(), a[4].cpu().numpy(), a[5].cpu().numpy()
        caps = packed[2].astype(np.int64) + packed[4].astype(np.int64)
        for q in range(npairs):
            for r in range(int(a[6][q].item())):
                o = poff[q] + r * caps[q]
                assert np.array_equal(pa[o:o + plen[q, r]], pb[o:o + plen[q, r]]), (q, r)
    s_ref, c_ref, f_ref = coopt.count_batch(*packed)
    assert np.array_equal(b[1].cpu().numpy().view(np.uint64), c_ref)


def test_center_star_argument_errors():
    L = nwp.lib()
    rng = np.random.default_rng(62)
    seqs = [random_seq(rng, int(rng.integers(30, 80))) for _ in range(6)]
    pool, off, lens = pack_seqs(seqs)
    d = [_dev(pool, np.uint8), _dev(off, np.int64), _dev(lens, np.int32)]
    ml = int(lens.max())
    S = nwp.allpairs(*d, ml)
    center = torch.zeros(1, dtype=torch.int32, device="cuda")
    width = torch.zeros(1, dtype=torch.int64, device="cuda")
    cap = int(lens.sum())
    msa = torch.empty((6, cap), dtype=torch.uint8, device="cuda")
    full = nwp.center_star_workspace_size(6, ml)
    ws = torch.empty(full, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream

    def call(nseq=6, wcap=cap, nbytes=full, maxl=ml):
        return L.nw_center_star(nseq, *[ptr(x) for x in d], maxl, P, ptr(S), 255, ptr(center), ptr(msa), wcap,
                                ptr(width), ptr(ws), nbytes, vp(st))

    assert call(wcap=-1) == nwp.NW_EINVAL
    assert call(nseq=-1) == nwp.NW_EINVAL
    assert call(nbytes=64) == nwp.NW_ENOSPC
    assert call(nseq=1 << 20, maxl=1 << 12) == nwp.NW_ERANGE
    assert call() == nwp.NW_OK
    torch.cuda.synchronize()
    assert int(width.item()) >= int(lens.max())
