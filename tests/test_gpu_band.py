"""Certified band: results bit-identical to the oracle (and to the full-grid
batch) for every starting half-width, with both growth rules (to the width a
failed pass's score certifies, and doubling) and the fallback exercised."""
import numpy as np
import pytest

import oracle
from oracle import band
from workloads import config_band_batch, pack_pairs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2412_21103_amd as nwp  # noqa: E402
from gpu_util import say  # noqa: E402

P = (1, -1, -1)


def _dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")


def run_band(pairs, w_init, scoring=P, w_default=0, frac=0.5, doubling=False, so=None):
    pool, ao, al, bo, bl = pack_pairs(pairs)
    ml = int(max(al.max(), bl.max()))
    wi = None if w_init is None else _dev(w_init, np.int32)
    s, paths, poff, plen, wu, st, cells = nwp.align_batch_banded(
        _dev(pool, np.uint8), _dev(ao, np.int64), _dev(al, np.int32), _dev(bo, np.int64),
        _dev(bl, np.int32), ml, scoring, w_init=wi, w_default=w_default, fallback_frac=frac,
        doubling=doubling, cells_score_only=so)
    torch.cuda.synchronize()
    paths = paths.cpu().numpy()
    poff = poff.cpu().numpy()
    plen = plen.cpu().numpy()
    out = [paths[poff[k]:poff[k] + plen[k]] for k in range(len(pairs))]
    return s.cpu().numpy(), out, wu.cpu().numpy(), st.cpu().numpy(), cells.cpu().numpy()


@pytest.fixture(scope="module")
def small_band_batch():
    pairs = config_band_batch(seed=77, npairs=48, lo=300, hi=2500)
    ref = [oracle.align(a, b, P) for a, b in zip(pairs.a, pairs.b)]
    return pairs, ref


def check_equal(pairs, ref, s, paths, tag):
    for k in range(len(pairs)):
        assert s[k] == ref[k][0], (tag, k, s[k], ref[k][0])
        assert paths[k].tolist() == ref[k][1].tolist(), (tag, k)


def test_band_with_certified_widths(small_band_batch):
    pairs, ref = small_band_batch
    wc = np.array([band.w_cert(r[0], len(a), len(b), P) for r, a, b in zip(ref, pairs.a, pairs.b)])
    say("band: w_init = w_cert")
    s, paths, wu, st, cells = run_band(pairs, wc)
    check_equal(pairs, ref, s, paths, "w_cert")
    # a start at w_cert certifies on the first pass, unless its band is past
    # the first pass's height limit (fallback_frac of m): then the first pass
    # runs the widest band under the limit and the second pass certifies
    m = np.array([len(a) for a in pairs.a])
    n = np.array([len(b) for b in pairs.b])
    limited = 128 + np.abs(n - m) + 2 * wc >= 0.5 * m
    first = (st & 1) == 1
    second = ((st >> 1) & 31) == 1
    fullg = (st & 0x40) != 0
    assert first[~limited].all()
    assert (first | second | fullg)[limited].all()
    assert first.sum() >= len(pairs) // 2


def test_band_doubling_from_zero(small_band_batch):
    pairs, ref = small_band_batch
    say("band: w_init = 0 (doubling)")
    so = torch.full((len(pairs),), -1, dtype=torch.int64, device="cuda")
    s, paths, wu, st, cells = run_band(pairs, None, w_default=0, doubling=True, so=so)
    check_equal(pairs, ref, s, paths, "w0=0")
    assert (so.cpu().numpy() == 0).all()  # doubling records directions on every pass
    doublings = (st >> 1) & 31
    assert doublings.max() >= 2
    # the certified width is never below the closed-form minimum
    for k in range(len(pairs)):
        if wu[k] >= 0:
            assert wu[k] >= band.w_cert(ref[k][0], len(pairs.a[k]), len(pairs.b[k]), P)


@pytest.mark.parametrize("w0", [0, 5, 40])
def test_band_widening_to_certified_width(small_band_batch, w0):
    # A failed pass widens the band to the width its own score certifies, so
    # the second pass always certifies (or is the full grid), and the final
    # width is at least w_cert.  The second pass records directions only in
    # a band around the first pass's; a path that leaves it costs the pass
    # again with directions in a band four times as wide (or everywhere).
    pairs, ref = small_band_batch
    say(f"band: w_init = {w0}, widening to the certified width")
    so = torch.full((len(pairs),), -1, dtype=torch.int64, device="cuda")
    s, paths, wu, st, cells = run_band(pairs, None, w_default=w0, so=so)
    check_equal(pairs, ref, s, paths, f"w0={w0}")
    # the first pass runs score-only unless it is the full grid: its cells are
    # counted there, and every later pass records directions
    so = so.cpu().numpy()
    fullg = (st & 0x40) != 0
    assert (so >= 0).all() and (so < cells).all()
    assert (so[~fullg] > 0).all()
    widenings = (st >> 1) & 31
    assert (widenings <= 4).all()
    if w0 == 0:
        assert (widenings[~fullg] >= 1).sum() > 0
    for k in range(len(pairs)):
        if wu[k] >= 0:
            assert wu[k] >= band.w_cert(ref[k][0], len(pairs.a[k]), len(pairs.b[k]), P)


def test_band_directions_only_in_first_band(small_band_batch):
    # After a failed first pass the certified band is swept with directions
    # only in a band 1.5 times as wide as the first pass's (+16).  Started at
    # each pair's own w_path (the oracle path's excursion), the path lies in
    # that band, so the walk never leaves it (at most two passes) -- unless
    # band(w_path) is past the first pass's height limit and the first pass
    # ran a narrower band; started at 0, paths with indels leave the
    # directions and take more passes.  Every path stays exact.
    pairs, ref = small_band_batch
    wp = np.array([band.w_path(r[1], len(a), len(b)) for r, a, b in zip(ref, pairs.a, pairs.b)])
    m = np.array([len(a) for a in pairs.a], np.int64)
    n = np.array([len(b) for b in pairs.b], np.int64)
    w_fb = (512 * m - 1024 * (128 + np.abs(n - m)) - 1) // 2048  # the first pass's limit at frac 0.5
    say("band: w_init = w_path")
    s, paths, wu, st, cells = run_band(pairs, wp)
    check_equal(pairs, ref, s, paths, "w_path")
    extra = (st >> 1) & 31
    assert (extra[wp <= w_fb] <= 1).all()
    assert (extra == 1).sum() > 0
    say("band: w_init = 0, walks that leave the straight band")
    s, paths, wu, st, cells = run_band(pairs, np.zeros(len(pairs), np.int64))
    check_equal(pairs, ref, s, paths, "zero")
    extra = (st >> 1) & 31
    assert (extra[wp <= 16] <= 1).all()
    assert (extra >= 2).sum() > 0


@pytest.mark.parametrize("start", ["w0=0", "w0=40", "w_path", "w_cert"])
def test_band_one_launch_same_outputs(small_band_batch, start):
    # With paths, the score-only first passes run in a launch of their own and
    # the launch with paths takes their results; every output (scores, paths,
    # widths, statuses, cells, score-only cells) equals that of the schedule
    # that runs all of a pair's passes in one launch.
    pairs, ref = small_band_batch
    if start.startswith("w0="):
        w_init, w_default = None, int(start[3:])
    else:
        f = band.w_path if start == "w_path" else None
        w_init = np.array([band.w_path(r[1], len(a), len(b)) if f else band.w_cert(r[0], len(a), len(b), P)
                           for r, a, b in zip(ref, pairs.a, pairs.b)])
        w_default = 0
    out = {}
    for one in (False, True):
        say(f"band: {start}, one launch = {one}")
        pool, ao, al, bo, bl = pack_pairs(pairs)
        ml = int(max(al.max(), bl.max()))
        so = torch.full((len(pairs),), -1, dtype=torch.int64, device="cuda")
        wi = None if w_init is None else _dev(w_init, np.int32)
        res = nwp.align_batch_banded(_dev(pool, np.uint8), _dev(ao, np.int64), _dev(al, np.int32),
                                     _dev(bo, np.int64), _dev(bl, np.int32), ml, P, w_init=wi,
                                     w_default=w_default, cells_score_only=so, one_launch=one)
        torch.cuda.synchronize()
        out[one] = [x.cpu().numpy() for x in res if x is not None] + [so.cpu().numpy()]
    # the paths buffer beyond each path's length is never written: compare paths
    for i, (x, y) in enumerate(zip(out[False], out[True])):
        if i != 1:
            assert np.array_equal(x, y), i
    s, paths, poff, plen = out[False][:4]
    paths1 = out[True][1]
    for k in range(len(pairs)):
        assert np.array_equal(paths[poff[k]:poff[k] + plen[k]], paths1[poff[k]:poff[k] + plen[k]]), k
    check_equal(pairs, ref, s, [paths[poff[k]:poff[k] + plen[k]] for k in range(len(pairs))], start)
    # the first passes that ran score-only are counted in the score-only cells
    st = out[False][5]
    assert (out[False][-1][(st & 0x40) == 0] > 0).all()


def test_band_forced_fallback(small_band_batch):
    pairs, ref = small_band_batch
    say("band: fallback fraction tiny -> full grid")
    s, paths, wu, st, cells = run_band(pairs, None, w_default=3, frac=1e-4)
    check_equal(pairs, ref, s, paths, "fallback")
    assert ((st & 0x40) != 0).all() and (wu == -1).all()
    m = np.array([len(a) for a in pairs.a], np.int64)
    n = np.array([len(b) for b in pairs.b], np.int64)
    assert (cells >= m * n).all()


def test_band_inapplicable_scoring():
    # 2*gap >= max(match, mismatch): the certificate does not apply, so the
    # band silently runs the full grid
    sc = (1, -1, 1)
    pairs = config_band_batch(seed=78, npairs=6, lo=200, hi=600)
    ref = [oracle.align(a, b, sc) for a, b in zip(pairs.a, pairs.b)]
    say("band: inapplicable scoring")
    s, paths, wu, st, cells = run_band(pairs, None, scoring=sc, w_default=2)
    check_equal(pairs, ref, s, paths, "inapplicable")
    assert ((st & 0x80) != 0).all()


def test_band_matches_full_batch(small_band_batch):
    pairs, ref = small_band_batch
    pool, ao, al, bo, bl = pack_pairs(pairs)
    ml = int(max(al.max(), bl.max()))
    say("band vs full batch, other scoring")
    sc = (2, -3, -2)
    s_full, paths_full, poff, plen = nwp.align_batch(
        _dev(pool, np.uint8), _dev(ao, np.int64), _dev(al, np.int32), _dev(bo, np.int64),
        _dev(bl, np.int32), ml, sc)
    torch.cuda.synchronize()
    s, paths, wu, st, cells = run_band(pairs, None, scoring=sc, w_default=8)
    assert (s == s_full.cpu().numpy()).all()
    pf = paths_full.cpu().numpy()
    po = poff.cpu().numpy()
    pl = plen.cpu().numpy()
    for k in range(len(pairs)):
        assert paths[k].tolist() == pf[po[k]:po[k] + pl[k]].tolist()


def test_band_empty_and_oversize_pairs():
    rng = np.random.default_rng(79)
    from workloads import Pairs, random_seq
    A = [random_seq(rng, m) for m in (0, 5, 0, 300, 40)]
    B = [random_seq(rng, n) for n in (0, 0, 7, 310, 45)]
    pairs = Pairs(A, B, "band_edges")
    ref = [oracle.align(a, b, P) for a, b in zip(A, B)]
    say("band: empty pairs")
    s, paths, wu, st, cells = run_band(pairs, np.array([3, 3, 3, 3, 3]))
    check_equal(pairs, ref, s, paths, "edges")
    for k in range(3):
        assert wu[k] == -1 and st[k] == 0x40 and cells[k] == 0, (k, wu[k], st[k], cells[k])
    # a pair longer than max_len is skipped with status 0
    pool, ao, al, bo, bl = pack_pairs(pairs)
    s2, _, _, pl, wu2, st2, cells2 = nwp.align_batch_banded(
        _dev(pool, np.uint8), _dev(ao, np.int64), _dev(al, np.int32), _dev(bo, np.int64),
        _dev(bl, np.int32), 100, P, w_default=2)
    torch.cuda.synchronize()
    s2, pl, wu2, st2, cells2 = (t.cpu().numpy() for t in (s2, pl, wu2, st2, cells2))
    assert s2[3] == np.iinfo(np.int32).min and pl[3] == -1
    assert wu2[3] == -1 and st2[3] == 0 and cells2[3] == 0
    assert s2[4] == ref[4][0]


@pytest.mark.parametrize("w0", [0, 1, 6])
def test_band_edge_shapes(w0):
    # Strip-boundary and ragged shapes through the band passes: the first pass
    # at a small width fails on mutated pairs, the second records directions
    # only in a narrow band (its three row ranges per strip empty or not,
    # depending on the shape and the sweep width), walks that leave it take
    # wider passes.  Every pair equals the oracle.
    rng = np.random.default_rng(80 + w0)
    from workloads import Pairs, mutate, random_seq
    lens = [1, 2, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 700, 1025]
    A, B = [], []
    for m in lens:
        for n in (m, max(1, m - 37), m + 41, max(1, m // 3)):
            a = random_seq(rng, m)
            b = mutate(rng, a, 0.2)[:n]
            if len(b) < n:
                b = np.concatenate([b, random_seq(rng, n - len(b))])
            A.append(a)
            B.append(b)
    pairs = Pairs(A, B, "band_shapes")
    ref = [oracle.align(a, b, P) for a, b in zip(A, B)]
    say(f"band: {len(A)} edge shapes from w0 = {w0}")
    s, paths, wu, st, cells = run_band(pairs, None, w_default=w0)
    check_equal(pairs, ref, s, paths, f"shapes w0={w0}")
    s, paths, wu, st, cells = run_band(pairs, None, w_default=w0, scoring=(2, -3, -2))
    ref2 = [oracle.align(a, b, (2, -3, -2)) for a, b in zip(A, B)]
    check_equal(pairs, ref2, s, paths, f"shapes w0={w0} other scoring")
