"""nw_autotune: measured sweep-width costs replace the built-in table; results
stay bit-exact (the table only changes which width each pass uses).  Every
sweep width, forced through the cost table, gives byte-identical results; a
measured table is kept in a JSON file keyed by architecture, compute-unit
count and config class, and installed from it in a later call."""
import numpy as np
import pytest

import oracle
from workloads import config_batch, pack_pairs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2412_21103_amd as nwp  # noqa: E402
from gpu_util import gpu_batch, say  # noqa: E402


def _dev(x, dt):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")


def test_autotune_then_exact():
    sample = config_batch(seed=71, npairs=256, lo=100, hi=2000)
    pool, ao, al, bo, bl = pack_pairs(sample)
    ml = int(max(al.max(), bl.max()))
    say("autotune on 256 pairs")
    table = nwp.autotune(_dev(pool, np.uint8), _dev(ao, np.int64), _dev(al, np.int32), _dev(bo, np.int64),
                         _dev(bl, np.int32), ml)
    say(f"autotune table {table}")
    assert table["dirs"][2] == 1000 and table["score"][2] == 1000
    assert all(c >= 1 for c in table["dirs"] + table["score"])
    try:
        pairs = config_batch(seed=72, npairs=120, lo=1, hi=1200)
        pool, ao, al, bo, bl = pack_pairs(pairs)
        s_ref, p_ref = oracle.align_batch(pool, ao, al, bo, bl, oracle.PAPER_SCORING)
        s, paths, _ = gpu_batch(pool, ao, al, bo, bl, int(max(al.max(), bl.max())))
        assert (s == s_ref).all()
        for k in range(len(pairs)):
            assert paths[k].tolist() == p_ref[k].tolist(), k
    finally:
        nwp.lib().nw_release_caches()


BIG = 1 << 20


@pytest.mark.parametrize("width", [128, 256, 512])
def test_every_sweep_width_gives_identical_results(width):
    # a cost table that leaves one width the only choice: each width must give
    # the oracle's scores and paths byte for byte (batch, banded, all-pairs)
    costs = {128: [1, BIG, BIG], 256: [BIG, 1, BIG], 512: [BIG, BIG, 1]}[width]
    pairs = config_batch(seed=73, npairs=80, lo=1, hi=1500)
    pool, ao, al, bo, bl = pack_pairs(pairs)
    ml = int(max(al.max(), bl.max()))
    s_ref, p_ref = oracle.align_batch(pool, ao, al, bo, bl, oracle.PAPER_SCORING)
    nwp.set_sweep_costs({"dirs": costs, "score": costs})
    try:
        table, tuned = nwp.sweep_costs()
        assert tuned and table["dirs"] == costs
        say(f"forced sweep width {width}")
        s, paths, _ = gpu_batch(pool, ao, al, bo, bl, ml)
        assert (s == s_ref).all()
        for k in range(len(pairs)):
            assert paths[k].tolist() == p_ref[k].tolist(), (width, k)
        d = [_dev(pool, np.uint8), _dev(ao, np.int64), _dev(al, np.int32), _dev(bo, np.int64), _dev(bl, np.int32)]
        out = nwp.align_batch_banded(*d, ml, w_default=16)
        torch.cuda.synchronize()
        sb, pb, ob, lb = (t.cpu().numpy() for t in out[:4])
        assert (sb == s_ref).all()
        for k in range(len(pairs)):
            assert pb[ob[k]:ob[k] + lb[k]].tolist() == p_ref[k].tolist(), (width, k)
        seqs = list(pairs.a[:24])
        from workloads import pack_seqs
        sp, so, sl = pack_seqs(seqs)
        from gpu_util import gpu_allpairs
        assert np.array_equal(gpu_allpairs(sp, so, sl, int(sl.max())), oracle.allpairs(sp, so, sl))
    finally:
        nwp.lib().nw_release_caches()
    assert nwp.sweep_costs()[1] is False


def test_autotune_table_kept_in_a_file(tmp_path):
    sample = config_batch(seed=74, npairs=128, lo=100, hi=2000)
    pool, ao, al, bo, bl = pack_pairs(sample)
    ml = int(max(al.max(), bl.max()))
    d = [_dev(pool, np.uint8), _dev(ao, np.int64), _dev(al, np.int32), _dev(bo, np.int64), _dev(bl, np.int32)]
    path = str(tmp_path / "autotune.json")
    try:
        table, measured = nwp.autotune_cached(path, *d, ml, config_class="batch_2000")
        assert measured and nwp.sweep_costs() == (table, True)
        nwp.lib().nw_release_caches()
        assert nwp.sweep_costs()[1] is False
        again, measured = nwp.autotune_cached(path, *d, ml, config_class="batch_2000")
        assert not measured and again == table and nwp.sweep_costs() == (table, True)
        import json
        keys = list(json.load(open(path)))
        assert len(keys) == 1 and keys[0].endswith("|batch_2000") and "|cu" in keys[0]
    finally:
        nwp.lib().nw_release_caches()
