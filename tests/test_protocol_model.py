"""CPU models of the hand-off protocols between waves, explored over random
interleavings: every wait ends (no deadlock) and every value a wave reads
was written by the strip it expects.

1. The cooperative long-pair fill: blocks of four waves take groups of four
   strips by atomic ticket (the grid smaller than the number of groups, so
   blocks come back for more); neighbouring waves of a block hand boundary
   rows over through an LDS ring with back-pressure (the writer overwrites a
   slot only once the row a ring length below has been read), the last wave
   of a block hands over to the next group's first wave through HBM slots
   with no back-pressure.  Group-end order as in the kernel: stores (after
   the room check), then the wait for the refill, then the consumed mark.

2. The co-optimal team fill: the four waves of a block sweep strips
   w, w+4, w+8, ... of one pair; strip s writes its last column to ring
   buffer s % 8 and publishes its progress there with tag s + 1; strip s+1
   waits for enough rows of that buffer.

Each model is a set of processes whose next action has a guard; a random
scheduler runs any process whose guard holds, and a state in which nothing
can run while some process is unfinished is a deadlock."""
import numpy as np
import pytest

GROUP = 32


def run_procs(procs, rng, max_actions=10_000_000):
    """Run generators that yield guards (callables); a process advances when
    its guard returns True.  Returns the number of actions taken."""
    pending = {i: next(p) for i, p in enumerate(procs)}
    taken = 0
    while pending:
        ready = [i for i, g in pending.items() if g()]
        assert ready, f"deadlock: {len(pending)} processes blocked"
        i = ready[int(rng.integers(len(ready)))]
        try:
            pending[i] = procs[i].send(None)
        except StopIteration:
            del pending[i]
        taken += 1
        assert taken < max_actions
    return taken


# ---------------------------------------------------------------- coop fill

def coop_model(m, nstrips, grid, ring, rng, room_check=True):
    ngroups_t = (nstrips + 3) // 4              # tickets (groups of four strips)
    ng = (m + 95) >> 5                          # sweep groups of one strip
    ticket = [0]
    stored = {}                                 # strip -> highest row stored for its reader
    consumed = {}                               # strip -> highest row its input ring reader has read
    lds_ring = {}                               # (block, reading wave) -> {slot: (writer strip, row)}
    block_state = {}                            # block -> [ticket, waves finished with it]
    reads = []

    def wave(b, w):
        while True:
            # __syncthreads; wave 0 takes the block's ticket, the rest see it
            st = block_state.setdefault(b, {"k": None, "done": 4, "epoch": 0})
            if w == 0:
                yield lambda: st["done"] == 4
                st["k"] = ticket[0]
                ticket[0] += 1
                st["done"] = 0
                st["epoch"] += 1
                for v in range(4):
                    lds_ring[(b, v)] = {}
            else:
                my_epoch = st.get("seen", {}).get(w, 0)
                yield lambda: st["epoch"] > my_epoch
                st.setdefault("seen", {})[w] = st["epoch"]
            k = st["k"]
            if k >= ngroups_t:
                st["done"] += 1
                return
            s = 4 * k + w
            if s >= nstrips:
                st["done"] += 1
                continue
            out_lds = (w < 3) and (s + 1 < nstrips)
            in_lds = (w > 0)
            stored[s] = 0
            consumed[s] = 0

            def have(r_hi):
                # rows 1..r_hi of the input are available
                r_hi = min(r_hi, m)
                if s == 0 or r_hi <= 0:
                    return True
                if in_lds:
                    ringb = lds_ring[(b, w)]
                    return all(ringb.get(r % ring) == (s - 1, r) for r in range(max(1, r_hi - GROUP + 1), r_hi + 1))
                return stored.get(s - 1, 0) >= r_hi

            def read(r_lo, r_hi):
                for r in range(max(1, r_lo), min(r_hi, m) + 1):
                    if s > 0:
                        if in_lds:
                            reads.append(lds_ring[(b, w)].get(r % ring) == (s - 1, r))
                        else:
                            reads.append(stored[s - 1] >= r)

            # first input rows 1..32
            yield lambda: have(GROUP)
            read(1, GROUP)
            for g in range(ng):
                # stores of rows 32g-63 .. 32g-32 after the room check
                r_hi = GROUP * g - GROUP
                if out_lds and room_check:
                    yield lambda r_hi=r_hi: consumed[s + 1] >= r_hi - ring if (s + 1) in consumed else r_hi <= ring
                lo, hi = max(1, r_hi - GROUP + 1), min(m, r_hi)
                for r in range(lo, hi + 1):
                    if out_lds:
                        lds_ring[(b, w + 1)][r % ring] = (s, r)
                if hi >= lo:
                    stored[s] = hi
                # the refill of rows 32g+33 .. 32g+64, then the consumed mark
                yield lambda g=g: have(GROUP * g + 2 * GROUP)
                read(GROUP * g + GROUP + 1, GROUP * g + 2 * GROUP)
                if in_lds:
                    consumed[s] = GROUP * g + 2 * GROUP
            st["done"] += 1

    procs = [wave(b, w) for b in range(grid) for w in range(4)]
    n = run_procs(procs, rng)
    assert all(reads), "a wave read a slot another strip had written"
    assert all(stored.get(s, 0) == m for s in range(nstrips - 1))
    return n


@pytest.mark.parametrize("m,nstrips,grid,ring", [
    (200, 9, 2, 1024), (1500, 13, 3, 1024), (3000, 8, 1, 1024), (3000, 16, 4, 1024),
    (700, 11, 2, 64), (700, 11, 3, 96), (2100, 7, 2, 128)])
def test_coop_fill_protocol(m, nstrips, grid, ring):
    rng = np.random.default_rng(m * 31 + nstrips)
    for _ in range(3):
        coop_model(m, nstrips, grid, ring, rng)


# ------------------------------------------------------- co-optimal team

def team_model(m, nstrips, rng, ring=8, waves=4, tagged=True):
    prog = [0] * ring                           # (tag << 32) | rows
    buf = [dict() for _ in range(ring)]         # row -> writer strip
    reads = []
    steps = m + 63

    def wave(w):
        for s in range(w, nstrips, waves):
            for T in range(0, steps, 64):
                if s > 0:
                    need = (s << 32) | min(T + 64, m)
                    if not tagged:  # progress compared without the strip tag
                        need &= 0xFFFFFFFF
                        yield lambda need=need: prog[(s - 1) % ring] & 0xFFFFFFFF >= need
                    else:
                        yield lambda need=need: prog[(s - 1) % ring] >= need
                    for r in range(T + 1, min(T + 64, m) + 1):
                        reads.append(buf[(s - 1) % ring].get(r) == s - 1)
                cnt = min(64, steps - T)
                if s + 1 < nstrips:
                    rows = min(m, max(0, T + cnt - 1 - 62))
                    for r in range(1, rows + 1):
                        buf[s % ring][r] = s
                    prog[s % ring] = ((s + 1) << 32) | rows
                    yield lambda: True

    run_procs([wave(w) for w in range(waves)], rng)
    assert all(reads), "a strip read a column its predecessor had not written"


@pytest.mark.parametrize("m,nstrips", [(1, 9), (64, 17), (130, 12), (700, 23), (2000, 9)])
def test_cooptimal_team_protocol(m, nstrips):
    rng = np.random.default_rng(m + nstrips)
    for _ in range(3):
        team_model(m, nstrips, rng)


def _fails(fn, tries=30):
    for _ in range(tries):
        try:
            fn()
        except AssertionError:
            return True
    return False


def test_models_catch_planted_mistakes():
    rng = np.random.default_rng(0)
    # progress read without its strip tag: a strip takes the column a strip
    # eight earlier left in the same ring buffer for its predecessor's
    assert _fails(lambda: team_model(700, 23, rng, tagged=False))
    # one ring buffer: a strip's own output passes for its predecessor's
    assert _fails(lambda: team_model(300, 9, rng, ring=1))
    # no room check on the LDS ring: the writer laps the reader
    assert _fails(lambda: coop_model(3000, 8, 2, 64, rng, room_check=False))
    # a ring shorter than the rows a refill takes in at once cannot hold them
    assert _fails(lambda: coop_model(700, 11, 2, 16, rng), tries=1)
