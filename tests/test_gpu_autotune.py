"""nw_autotune: measured sweep-width costs replace the built-in table; results
stay bit-exact (the table only changes which width each pass uses)."""
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
