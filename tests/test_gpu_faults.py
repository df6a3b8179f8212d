"""Device-fault reporting, forced from the host; nw_align under graph capture
and on reused workspace memory.

The waits between waves are bounded; nw_set_wait_limit makes them give up
after a few polls so that the failure path runs without any real fault: every
kernel drains and exits normally, the outputs carry the failure values, and
the next call (or nw_sync) reports NW_EDEVICE.  The limit is restored before
each test ends, and a normal call afterwards must be exact again.

Graph capture: nw_align on a pair wide enough for the multi-wave engine is
captured once and replayed, with the input bytes changed in place between
replays and eager work in between; every replay must equal the oracle on the
bytes it read.  Reused memory: stale slots and header words in a workspace
never pass for a later call's data."""
import numpy as np
import pytest

import oracle
from workloads import config_batch, mutate, pack_pairs, random_seq

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2412_21103_amd as nwp  # noqa: E402
from gpu_util import dev_u8, say  # noqa: E402

INT32_MIN = -(2 ** 31)


def _pair(seed, m):
    rng = np.random.default_rng(seed)
    a = random_seq(rng, m)
    return a, mutate(rng, a, 0.1)


def _exact(a, b, s, path, plen):
    s_ref, p_ref = oracle.align(a, b)
    k = int(plen.item())
    return int(s.item()) == s_ref and k == len(p_ref) and path[:k].cpu().numpy().tolist() == p_ref.tolist()


@pytest.mark.parametrize("walk", [1 << 30, 1], ids=["one_wave_walk", "strip_parallel_walk"])
def test_wait_limit_reports_fault_and_recovers(walk):
    a, b = _pair(1, 4096)  # 32 strips on 8 blocks: waits inside blocks and between them
    da, db = dev_u8(a), dev_u8(b)
    say(f"faults: nw_align with a wait limit of one poll, walk limit {walk}")
    nwp.set_wait_limit(1)
    nwp.set_walk_limit(walk)
    try:
        s, path, plen = nwp.align(da, db)
        with pytest.raises(nwp.NWError) as e:
            nwp.sync()
        assert e.value.status == -4
        assert int(s.item()) == INT32_MIN and int(plen.item()) == -3
        # reported once: a second sync is clean
        nwp.sync()
        # the fault also surfaces at the next call when nobody called nw_sync
        s, path, plen = nwp.align(da, db, score_only=True)
        torch.cuda.synchronize()
        assert int(s.item()) == INT32_MIN
        with pytest.raises(nwp.NWError) as e:
            nwp.align(da, db)
        assert e.value.status == -4
        nwp.set_wait_limit(0)
        say("faults: default wait limit again")
        s, path, plen = nwp.align(da, db)
        nwp.sync()
        assert _exact(a, b, s, path, plen)
    finally:
        nwp.set_wait_limit(0)
        nwp.set_walk_limit(0)


def test_wait_limit_cooptimal_teams():
    pairs = config_batch(seed=77, npairs=12, lo=600, hi=900)  # >= 2^16 cells: filled by teams
    pool, ao, al, bo, bl = pack_pairs(pairs)
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")
    d = [dev_u8(pool), t(ao, np.int64), t(al, np.int32), t(bo, np.int64), t(bl, np.int32)]
    max_len = int(max(al.max(), bl.max()))
    say("faults: co-optimal team waits with a limit of one poll")
    nwp.set_wait_limit(1)
    try:
        out = nwp.cooptimal(*d, max_len, nwp.PAPER_SCORING)
        with pytest.raises(nwp.NWError) as e:
            nwp.sync()
        assert e.value.status == -4
        s = out[0].cpu().numpy()
        assert (s == INT32_MIN).any()
    finally:
        nwp.set_wait_limit(0)
    out = nwp.cooptimal(*d, max_len, nwp.PAPER_SCORING)
    nwp.sync()
    s_ref = np.array([oracle.score(x, y) for x, y in zip(pairs.a, pairs.b)])
    assert (out[0].cpu().numpy() == s_ref).all()


def test_set_wait_limit_rejects_negative():
    assert nwp.lib().nw_set_wait_limit(-1) == -1
    assert nwp.lib().nw_set_walk_limit(-1) == -1


def test_align_graph_replays_see_new_inputs():
    m = 3000
    a0, b0 = _pair(2, m)
    n = len(b0)
    da, db = dev_u8(a0), dev_u8(b0)
    ws = torch.empty(nwp.align_workspace_size(m, n, 0), dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        nwp.align(da, db, workspace=ws)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say("faults: capturing nw_align into a graph")
    with torch.cuda.graph(g):
        s, path, plen = nwp.align(da, db, workspace=ws)
    rng = np.random.default_rng(3)
    for r in range(4):
        if r == 0:
            a, b = a0, b0
        else:
            a = random_seq(rng, m)
            b = mutate(rng, a, 0.05 * r)[:n]
            if len(b) < n:
                b = np.concatenate([b, random_seq(rng, n - len(b))])
            da.copy_(dev_u8(a))
            db.copy_(dev_u8(b))
        g.replay()
        torch.cuda.synchronize()
        assert _exact(a, b, s, path, plen), r
        # eager work on the same workspace between replays
        s2, p2, l2 = nwp.align(da, db, workspace=ws)
        torch.cuda.synchronize()
        assert _exact(a, b, s2, p2, l2), r


def test_align_reused_workspace_with_stale_contents():
    # A workspace is reused memory: boundary slots and header words that any
    # earlier call left in it must never pass for this call's data.  One
    # workspace, new input bytes every call, the header region overwritten
    # between calls (random words, and words copied from the slot area, which
    # hold earlier calls' tags), eager calls interleaved with graph replays.
    m = 2500
    rng = np.random.default_rng(11)
    a0 = random_seq(rng, m)
    b0 = mutate(rng, a0, 0.1)
    n = len(b0)
    da, db = dev_u8(a0), dev_u8(b0)
    ws = torch.empty(nwp.align_workspace_size(m, n, 0), dtype=torch.uint8, device="cuda")
    nwp.align(da, db, workspace=ws)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    say("faults: reused workspace with stale header and slots")
    with torch.cuda.graph(g):
        gs, gpath, gplen = nwp.align(da, db, workspace=ws)
    hdr = ws[:256]
    for r in range(12):
        a = random_seq(rng, m)
        b = mutate(rng, a, 0.02 + 0.02 * (r % 5))[:n]
        if len(b) < n:
            b = np.concatenate([b, random_seq(rng, n - len(b))])
        da.copy_(dev_u8(a))
        db.copy_(dev_u8(b))
        if r % 3 == 0:
            hdr.copy_(torch.from_numpy(rng.integers(0, 256, 256, dtype=np.uint8)).cuda())
        elif r % 3 == 1:
            hdr.copy_(ws[256 + 64 * r:512 + 64 * r])
        if r % 2 == 0:
            s, path, plen = nwp.align(da, db, workspace=ws)
        else:
            g.replay()
            s, path, plen = gs, gpath, gplen
        torch.cuda.synchronize()
        assert _exact(a, b, s, path, plen), r
