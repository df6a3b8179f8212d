"""NW_GRAPH: the batch entry points captured into a HIP graph and replayed.

Every replay is checked against an eager call on the same inputs, with other
eager GPU work and synchronisations between replays, and with the input bytes
changed in place between replays (a replay must read the current inputs)."""
import ctypes

import numpy as np
import pytest

from workloads import config_band_batch, config_batch, pack_pairs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2412_21103_amd as nwp  # noqa: E402
from gpu_util import say  # noqa: E402

NW_GRAPH = 0x2
vp = ctypes.c_void_p


def _dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")


class BatchBuffers:
    def __init__(self, pairs):
        pool, ao, al, bo, bl = pack_pairs(pairs)
        self.n = len(pairs)
        self.max_len = int(max(al.max(), bl.max()))
        self.pool = _dev(pool, np.uint8)
        self.ao, self.al = _dev(ao, np.int64), _dev(al, np.int32)
        self.bo, self.bl = _dev(bo, np.int64), _dev(bl, np.int32)
        caps = al.astype(np.int64) + bl
        self.poff = _dev(np.concatenate([[0], np.cumsum(caps)[:-1]]), np.int64)
        self.total = int(caps.sum())

    def outputs(self):
        return (torch.empty(self.n, dtype=torch.int32, device="cuda"),
                torch.empty(self.total, dtype=torch.uint8, device="cuda"),
                torch.empty(self.n, dtype=torch.int32, device="cuda"))

    def ins(self):
        p = lambda t: vp(t.data_ptr())
        return [p(self.pool), p(self.ao), p(self.al), p(self.bo), p(self.bl)]


def _paths(out, B):
    s, paths, plen = (t.cpu().numpy() for t in out)
    poff = B.poff.cpu().numpy()
    return s, [paths[poff[k]:poff[k] + plen[k]].tolist() for k in range(B.n)]


def _batch(B, out, ws, flags, stream):
    s, paths, plen = out
    p = lambda t: vp(t.data_ptr())
    return nwp.lib().nw_align_batch(B.n, *B.ins(), B.max_len, nwp.Scoring(1, -1, -1), flags, p(s), p(paths),
                                    p(B.poff), p(plen), p(ws), ws.numel(), vp(stream.cuda_stream))


def _banded(B, out, extra, ws, flags, stream):
    s, paths, plen = out
    w_used, status, cells = extra
    p = lambda t: vp(t.data_ptr())
    return nwp.lib().nw_align_batch_banded(B.n, *B.ins(), B.max_len, nwp.Scoring(1, -1, -1), flags, None, 4,
                                           ctypes.c_float(0.5), p(s), p(paths), p(B.poff), p(plen),
                                           p(w_used), p(status), p(cells), vp(0), p(ws), ws.numel(),
                                           vp(stream.cuda_stream))


def test_graph_replays_match_eager():
    pairs = config_batch(seed=61, npairs=96, lo=50, hi=900)
    other = config_batch(seed=62, npairs=96, lo=50, hi=900)
    B = BatchBuffers(pairs)
    ws = torch.empty(nwp.batch_workspace_size(B.n, B.max_len), dtype=torch.uint8, device="cuda")
    ws_e = torch.empty_like(ws)
    g_out, e_out = B.outputs(), B.outputs()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        assert _batch(B, g_out, ws, NW_GRAPH, torch.cuda.default_stream()) == nwp.NW_EINVAL  # null stream
        for rep in range(4):
            say(f"graph: batch replay {rep}")
            if rep == 2:
                # new sequence bytes of the same lengths, written in place
                pool2 = np.concatenate([np.concatenate([a, b]) for a, b in zip(other.a, other.b)])
                al = np.array([len(a) for a in pairs.a])
                if (al == np.array([len(a) for a in other.a])).all():
                    B.pool.copy_(_dev(pool2, np.uint8))
                else:
                    B.pool.copy_(torch.flip(B.pool, [0]))
            assert _batch(B, e_out, ws_e, 0, st) == 0
            assert _batch(B, g_out, ws, NW_GRAPH, st) == 0
            # unrelated eager work between replays
            junk = torch.randn(1 << 20, device="cuda").cumsum(0)
            st.synchronize()
            torch.cuda.synchronize()
            assert float(junk[-1].item()) == float(junk[-1].item())
            eg, ee = _paths(g_out, B), _paths(e_out, B)
            assert (eg[0] == ee[0]).all(), rep
            assert eg[1] == ee[1], rep
            for t in g_out:
                t.fill_(0x5A if t.dtype == torch.uint8 else -7)


def test_banded_graph_replays_match_eager():
    pairs = config_band_batch(seed=63, npairs=40, lo=200, hi=1500)
    B = BatchBuffers(pairs)
    ws = torch.empty(nwp.banded_workspace_size(B.n, B.max_len), dtype=torch.uint8, device="cuda")
    ws_e = torch.empty_like(ws)
    g_out, e_out = B.outputs(), B.outputs()
    mk = lambda: (torch.empty(B.n, dtype=torch.int32, device="cuda"), torch.empty(B.n, dtype=torch.uint8, device="cuda"),
                  torch.empty(B.n, dtype=torch.int64, device="cuda"))
    g_x, e_x = mk(), mk()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for rep in range(4):
            say(f"graph: banded replay {rep}")
            if rep == 2:
                # new bytes in place (same lengths): the replay's first passes
                # find other scores, and its pairs are ordered again on the device
                B.pool.copy_(torch.flip(B.pool, [0]))
            assert _banded(B, e_out, e_x, ws_e, 0, st) == 0
            assert _banded(B, g_out, g_x, ws, NW_GRAPH, st) == 0
            # unrelated eager work between replays
            junk = torch.randn(1 << 20, device="cuda").cumsum(0)
            st.synchronize()
            torch.cuda.synchronize()
            assert float(junk[-1].item()) == float(junk[-1].item())
            eg, ee = _paths(g_out, B), _paths(e_out, B)
            assert (eg[0] == ee[0]).all() and eg[1] == ee[1], rep
            for a, b in zip(g_x, e_x):
                assert torch.equal(a, b), rep
            for t in g_out + g_x:
                t.fill_(3)
    nwp.lib().nw_release_caches()
