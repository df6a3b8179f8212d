"""The C-ABI library loads, exports every function include/nw.h declares, and
rejects bad arguments on the host (no GPU needed for any of this)."""
import ctypes
import subprocess

import pytest

nwp = pytest.importorskip("paper_2412_21103_amd")


def test_exports_every_declared_function():
    declared = nwp.declared_functions()
    assert {"nw_align", "nw_align_batch", "nw_allpairs_scores", "nw_strerror"} <= set(declared)
    out = subprocess.run(["nm", "-D", "--defined-only", nwp._LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [f for f in declared if f not in exported]
    assert not missing, missing
    L = nwp.lib()
    for f in declared:
        assert hasattr(L, f)


def test_strerror_and_version():
    L = nwp.lib()
    for st in [0, -1, -2, -3, -4, -5, 7]:
        assert isinstance(L.nw_strerror(st), bytes)
    assert L.nw_version() >= 100


def _align(**kw):
    args = dict(a=1, m=4, b=1, n=4, sc=nwp.Scoring(1, -1, -1), flags=0, score=1, path=1, cap=8,
                plen=1, ws=1, wsb=1 << 30, stream=None)
    args.update(kw)
    vp = ctypes.c_void_p
    return nwp.lib().nw_align(vp(args["a"]), args["m"], vp(args["b"]), args["n"], args["sc"],
                              args["flags"], vp(args["score"]), vp(args["path"]), args["cap"],
                              vp(args["plen"]), vp(args["ws"]), args["wsb"], vp(args["stream"]))


def test_host_argument_checks():
    # every one of these is rejected before any HIP call
    assert _align(m=-1) == nwp.NW_EINVAL
    assert _align(a=0) == nwp.NW_EINVAL
    assert _align(b=0) == nwp.NW_EINVAL
    assert _align(score=0) == nwp.NW_EINVAL
    assert _align(plen=0) == nwp.NW_EINVAL
    assert _align(ws=0) == nwp.NW_EINVAL
    assert _align(cap=7) == nwp.NW_ENOSPC
    assert _align(flags=0x80) == nwp.NW_EINVAL
    # diagonal term 4*(s - 2 gap) + 2 at or beyond 2^22 (terms beyond a
    # signed byte alone are legal: they take the byte-comparing sweep)
    assert _align(sc=nwp.Scoring(1 << 20, -1, -1)) == nwp.NW_ERANGE
    # overflow guard on lengths
    assert _align(m=1 << 27, n=1 << 27, cap=1 << 28) == nwp.NW_ERANGE
    vp = ctypes.c_void_p
    L = nwp.lib()
    assert L.nw_align_batch(-1, vp(1), vp(1), vp(1), vp(1), vp(1), 10, nwp.Scoring(1, -1, -1), 0,
                            vp(1), vp(1), vp(1), vp(1), vp(1), 1, vp(0)) == nwp.NW_EINVAL
    assert L.nw_align_batch(4, vp(0), vp(1), vp(1), vp(1), vp(1), 10, nwp.Scoring(1, -1, -1), 0,
                            vp(1), vp(1), vp(1), vp(1), vp(1), 1, vp(0)) == nwp.NW_EINVAL
    assert L.nw_align_batch(4, vp(1), vp(1), vp(1), vp(1), vp(1), 10, nwp.Scoring(1, -1, -1), 0,
                            vp(1), vp(0), vp(1), vp(1), vp(1), 1, vp(0)) == nwp.NW_EINVAL
    assert L.nw_align_batch(0, vp(0), vp(0), vp(0), vp(0), vp(0), 10, nwp.Scoring(1, -1, -1), 0,
                            vp(0), vp(0), vp(0), vp(0), vp(0), 0, vp(0)) == nwp.NW_OK
    # graph replay needs a real stream; unknown flag bits are rejected
    assert L.nw_align_batch(4, vp(1), vp(1), vp(1), vp(1), vp(1), 10, nwp.Scoring(1, -1, -1), nwp.GRAPH,
                            vp(1), vp(1), vp(1), vp(1), vp(1), 1 << 30, vp(0)) == nwp.NW_EINVAL
    assert L.nw_align_batch(4, vp(1), vp(1), vp(1), vp(1), vp(1), 10, nwp.Scoring(1, -1, -1), 0x4,
                            vp(1), vp(1), vp(1), vp(1), vp(1), 1 << 30, vp(1)) == nwp.NW_EINVAL
    L.nw_release_caches()
    assert L.nw_allpairs_scores(-3, vp(1), vp(1), vp(1), 10, nwp.Scoring(1, -1, -1), vp(1), vp(1), 1,
                                vp(0)) == nwp.NW_EINVAL
    assert L.nw_allpairs_scores(70000, vp(1), vp(1), vp(1), 10, nwp.Scoring(1, -1, -1), vp(1), vp(1),
                                1, vp(0)) == nwp.NW_ERANGE


def test_band_model_host_checks():
    vp = ctypes.c_void_p
    L = nwp.lib()
    P = nwp.Scoring(1, -1, -1)
    sz = ctypes.c_size_t(0)
    assert L.nw_mlp_train_workspace_size(0, ctypes.byref(sz)) == nwp.NW_EINVAL
    assert L.nw_mlp_train_workspace_size(256, ctypes.byref(sz)) == nwp.NW_OK
    assert sz.value >= (3 * 256 + 4 * 256 * 64 + 9 * nwp.MLP_PARAMS) * 4
    # labels need an applicable certificate: 2*gap < max(match, mismatch)
    assert L.nw_band_labels(4, vp(1), vp(1), vp(1), nwp.Scoring(1, -1, 1), vp(1), vp(1), vp(0)) == nwp.NW_EINVAL
    assert L.nw_band_labels(-1, vp(1), vp(1), vp(1), P, vp(1), vp(1), vp(0)) == nwp.NW_EINVAL
    assert L.nw_band_labels(0, vp(0), vp(0), vp(0), P, vp(0), vp(0), vp(0)) == nwp.NW_OK
    assert L.nw_band_labels(4, vp(1), vp(1), vp(1), P, vp(0), vp(0), vp(0)) == nwp.NW_EINVAL
    # missing model arrays, bad tau, bad lr, empty batch, short workspace
    st = nwp.MlpState(0, 0, 0, 0, 0)
    assert L.nw_mlp_forward(ctypes.byref(st), 4, vp(1), vp(1), vp(0)) == nwp.NW_EINVAL
    assert L.nw_mlp_sync(ctypes.byref(st), vp(0)) == nwp.NW_EINVAL
    ok = nwp.MlpState(1, 1, 1, 1, 0)
    f = ctypes.c_float
    step = L.nw_mlp_train_step
    assert step(ctypes.byref(ok), 8, vp(1), vp(1), vp(0), f(1.0), f(1e-3), vp(0), vp(0), vp(1), 1 << 30, vp(0)) == nwp.NW_EINVAL
    assert step(ctypes.byref(ok), 8, vp(1), vp(1), vp(0), f(0.9), f(-1.0), vp(0), vp(0), vp(1), 1 << 30, vp(0)) == nwp.NW_EINVAL
    assert step(ctypes.byref(ok), 0, vp(1), vp(1), vp(0), f(0.9), f(1e-3), vp(0), vp(0), vp(1), 1 << 30, vp(0)) == nwp.NW_EINVAL
    assert step(ctypes.byref(ok), 8, vp(1), vp(1), vp(0), f(0.9), f(1e-3), vp(0), vp(0), vp(1), 16, vp(0)) == nwp.NW_ENOSPC
    no_adam = nwp.MlpState(1, 1, 0, 0, 0)
    assert step(ctypes.byref(no_adam), 8, vp(1), vp(1), vp(0), f(0.9), f(1e-3), vp(0), vp(0), vp(1), 1 << 30, vp(0)) == nwp.NW_EINVAL
    assert L.nw_mlp_train_epoch(ctypes.byref(ok), 8, vp(1), vp(1), vp(0), 4, f(0.9), f(1e-3), vp(0), vp(1),
                                1 << 30, vp(0)) == nwp.NW_EINVAL
    assert L.nw_mlp_widths(4, vp(1), vp(1), vp(1), f(-0.5), vp(1), vp(0)) == nwp.NW_EINVAL
    assert L.nw_mlp_widths(0, vp(0), vp(0), vp(0), f(0.1), vp(0), vp(0)) == nwp.NW_OK
    assert L.nw_mlp_features(-2, vp(1), vp(1), vp(1), vp(1), vp(1), vp(1), vp(0)) == nwp.NW_EINVAL
    assert L.nw_align_batch_learned(4, vp(1), vp(1), vp(1), vp(1), vp(1), 10, P, 0, ctypes.byref(st),
                                    f(0.1), f(0.5), vp(1), vp(1), vp(1), vp(1), vp(0), vp(0), vp(0),
                                    vp(0), vp(1), 1 << 30, vp(0)) == nwp.NW_EINVAL


def test_flag_constants_match_header():
    # the binding's flag values are the header's #defines
    import re
    text = open(nwp._HEADER).read()
    defs = {k: int(v, 16) for k, v in re.findall(r"#define NW_([A-Z_]+) 0x([0-9a-fA-F]+)u", text)}
    assert defs == {"SCORE_ONLY": nwp.SCORE_ONLY, "GRAPH": nwp.GRAPH, "BAND_DOUBLING": nwp.BAND_DOUBLING,
                    "BAND_ONE_LAUNCH": nwp.BAND_ONE_LAUNCH}
    # flags are distinct bits
    vals = list(defs.values())
    assert all(v & (v - 1) == 0 for v in vals) and len(set(vals)) == len(vals)
