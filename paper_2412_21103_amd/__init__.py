"""Python binding for libnw (Needleman-Wunsch with a linear gap on MI355X).

Argument marshalling only: every step of the alignment runs in the HIP
kernels of ``libnw.so``.  Tensors must be CUDA (HIP) tensors on the current
device; work is queued on torch's current stream unless ``stream`` is given.
The library must have been built (``__graft_entry__.build()``); importing
this package without it raises ImportError.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

__all__ = [
    "Scoring", "NWError", "PAPER_SCORING", "lib", "align", "align_batch", "allpairs",
    "align_workspace_size", "batch_workspace_size", "allpairs_workspace_size",
    "declared_functions", "MOVE_D", "MOVE_U", "MOVE_L", "SCORE_ONLY", "GRAPH", "profile_begin",
    "profile_end", "align_batch_banded", "banded_workspace_size", "Mlp", "MLP_INPUTS",
    "MLP_PARAMS", "mlp_features", "mlp_forward", "mlp_widths", "band_labels", "path_labels", "mlp_train_step",
    "mlp_train_epoch", "align_batch_learned", "learned_workspace_size", "autotune", "init", "sync",
    "set_wait_limit", "set_walk_limit", "align_noalloc", "align_noalloc_fits", "sweep_costs", "set_sweep_costs",
    "autotune_cached",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libnw.so")
_HEADER = os.path.join(os.path.dirname(_HERE), "include", "nw.h")

MOVE_D, MOVE_U, MOVE_L = 1, 2, 3
SCORE_ONLY = 0x1
GRAPH = 0x2
BAND_DOUBLING = 0x4
BAND_ONE_LAUNCH = 0x8
PAPER_SCORING = (1, -1, -1)

NW_OK, NW_EINVAL, NW_ERANGE, NW_ENOSPC, NW_EDEVICE, NW_ENOTSUP = 0, -1, -2, -3, -4, -5
MLP_INPUTS, MLP_HIDDEN, MLP_PARAMS = 259, 64, 20865


class Scoring(ctypes.Structure):
    _fields_ = [("match", ctypes.c_int32), ("mismatch", ctypes.c_int32), ("gap", ctypes.c_int32)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_int32), ("total_ms", ctypes.c_double)]


class MlpState(ctypes.Structure):
    _fields_ = [("params", ctypes.c_void_p), ("params_bf16", ctypes.c_void_p),
                ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p), ("step", ctypes.c_int64)]


class NWError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {lib().nw_strerror(status).decode()} (status {status})")


_lib = None
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_sz = ctypes.c_size_t


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(_LIB_PATH)
        L.nw_strerror.argtypes = [ctypes.c_int]
        L.nw_strerror.restype = ctypes.c_char_p
        L.nw_version.restype = ctypes.c_int
        L.nw_align_workspace_size.argtypes = [_i64, _i64, _u32, ctypes.POINTER(_sz)]
        L.nw_align.argtypes = [_vp, _i64, _vp, _i64, Scoring, _u32, _vp, _vp, _i64, _vp, _vp, _sz, _vp]
        L.nw_align_noalloc.argtypes = [_vp, _i64, _vp, _i64, Scoring, _u32, _vp, _vp, _i64, _vp, _vp]
        L.nw_align_noalloc_fits.argtypes = [_i64, _i64, _u32]
        L.nw_align_batch_workspace_size.argtypes = [_i32, _i32, _u32, ctypes.POINTER(_sz)]
        L.nw_align_batch.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _i32, Scoring, _u32, _vp, _vp,
                                     _vp, _vp, _vp, _sz, _vp]
        L.nw_align_batch_banded_workspace_size.argtypes = [_i32, _i32, _u32, ctypes.POINTER(_sz)]
        L.nw_align_batch_banded.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _i32, Scoring, _u32, _vp,
                                            _i32, ctypes.c_float, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                            _vp, _vp, _sz, _vp]
        _pm = ctypes.POINTER(MlpState)
        _f = ctypes.c_float
        L.nw_mlp_sync.argtypes = [_pm, _vp]
        L.nw_mlp_features.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.nw_mlp_forward.argtypes = [_pm, _i32, _vp, _vp, _vp]
        L.nw_mlp_widths.argtypes = [_i32, _vp, _vp, _vp, _f, _vp, _vp]
        L.nw_band_labels.argtypes = [_i32, _vp, _vp, _vp, Scoring, _vp, _vp, _vp]
        L.nw_path_labels.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]
        L.nw_mlp_train_workspace_size.argtypes = [_i32, ctypes.POINTER(_sz)]
        L.nw_mlp_train_step.argtypes = [_pm, _i32, _vp, _vp, _vp, _f, _f, _vp, _vp, _vp, _sz, _vp]
        L.nw_mlp_train_epoch.argtypes = [_pm, _i32, _vp, _vp, _vp, _i32, _f, _f, _vp, _vp, _sz, _vp]
        L.nw_align_batch_learned_workspace_size.argtypes = [_i32, _i32, _u32, ctypes.POINTER(_sz)]
        L.nw_align_batch_learned.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _i32, Scoring, _u32, _pm,
                                             _f, _f, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _sz, _vp]
        L.nw_autotune.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp, _sz, _vp, _vp]
        L.nw_allpairs_workspace_size.argtypes = [_i32, _i32, ctypes.POINTER(_sz)]
        L.nw_allpairs_scores.argtypes = [_i32, _vp, _vp, _vp, _i32, Scoring, _vp, _vp, _sz, _vp]
        L.nw_center_star_workspace_size.argtypes = [_i32, _i32, ctypes.POINTER(_sz)]
        L.nw_center_star.argtypes = [_i32, _vp, _vp, _vp, _i32, Scoring, _vp, ctypes.c_uint8, _vp, _vp, _i64,
                                     _vp, _vp, _sz, _vp]
        L.nw_cooptimal_workspace_size.argtypes = [_i32, _i32, _i32, ctypes.POINTER(_sz)]
        L.nw_cooptimal.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _i32, Scoring, _vp, _vp, _vp, _i32, _vp, _vp,
                                   _vp, _vp, _vp, _sz, _vp]
        L.nw_init.restype = ctypes.c_int
        L.nw_sync.argtypes = [_vp]
        L.nw_sync.restype = ctypes.c_int
        L.nw_set_wait_limit.argtypes = [_i32]
        L.nw_set_wait_limit.restype = ctypes.c_int
        L.nw_set_walk_limit.argtypes = [ctypes.c_int64]
        L.nw_set_walk_limit.restype = ctypes.c_int
        L.nw_release_caches.restype = None
        L.nw_sweep_costs.argtypes = [_vp, _vp]
        L.nw_set_sweep_costs.argtypes = [_vp]
        L.nw_profile_begin.restype = ctypes.c_int
        L.nw_profile_end.argtypes = [ctypes.POINTER(KernelTime), _i32, ctypes.POINTER(_i32)]
        _lib = L
    return _lib


def declared_functions():
    """Names of the functions include/nw.h declares."""
    text = open(_HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nw_[a-z_0-9]+)\s*\(", text)))


def _check(st: int, where: str):
    if st != NW_OK:
        raise NWError(st, where)


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else _vp(0)


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


def _sc(scoring):
    if isinstance(scoring, Scoring):
        return scoring
    return Scoring(*[int(x) for x in scoring])


def _dev():
    return torch.device("cuda", torch.cuda.current_device())


def align_workspace_size(m: int, n: int, flags: int = 0) -> int:
    out = _sz(0)
    _check(lib().nw_align_workspace_size(int(m), int(n), int(flags), ctypes.byref(out)), "nw_align_workspace_size")
    return int(out.value)


def batch_workspace_size(npairs: int, max_len: int, flags: int = 0) -> int:
    out = _sz(0)
    _check(lib().nw_align_batch_workspace_size(int(npairs), int(max_len), int(flags), ctypes.byref(out)),
           "nw_align_batch_workspace_size")
    return int(out.value)


def allpairs_workspace_size(nseq: int, max_len: int) -> int:
    out = _sz(0)
    _check(lib().nw_allpairs_workspace_size(int(nseq), int(max_len), ctypes.byref(out)),
           "nw_allpairs_workspace_size")
    return int(out.value)


def _workspace(nbytes, workspace):
    if workspace is not None and workspace.numel() >= nbytes:
        return workspace
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=_dev())


def align(a: torch.Tensor, b: torch.Tensor, scoring=PAPER_SCORING, score_only: bool = False,
          workspace: torch.Tensor | None = None, stream=None):
    """Align one pair.  Returns ``(score, path, path_len)`` device tensors:
    int32[1], uint8[m+n] (moves from (0,0); only the first path_len are set)
    and int64[1].  ``path`` and ``path_len`` are None with ``score_only``."""
    m, n = int(a.numel()), int(b.numel())
    flags = SCORE_ONLY if score_only else 0
    dev = _dev()
    ws = _workspace(align_workspace_size(m, n, flags), workspace)
    score = torch.empty(1, dtype=torch.int32, device=dev)
    path = None if score_only else torch.empty(max(m + n, 1), dtype=torch.uint8, device=dev)
    plen = None if score_only else torch.empty(1, dtype=torch.int64, device=dev)
    st = lib().nw_align(_ptr(a), m, _ptr(b), n, _sc(scoring), flags, _ptr(score), _ptr(path),
                        (m + n) if path is not None else 0, _ptr(plen), _ptr(ws), ws.numel(),
                        _stream(stream))
    _check(st, "nw_align")
    return score, path, plen


def align_noalloc(a: torch.Tensor, b: torch.Tensor, score: torch.Tensor, path: torch.Tensor | None = None,
                  path_len: torch.Tensor | None = None, scoring=PAPER_SCORING, stream=None):
    """nw_align on the library's own fixed device scratch: the caller passes
    the outputs (int32[1] score; uint8[>= m+n] path and int64[1] path_len, or
    None for the score only) and the call allocates nothing."""
    m, n = int(a.numel()), int(b.numel())
    flags = SCORE_ONLY if path is None else 0
    cap = int(path.numel()) if path is not None else 0
    st = lib().nw_align_noalloc(_ptr(a), m, _ptr(b), n, _sc(scoring), flags, _ptr(score), _ptr(path), cap,
                                _ptr(path_len), _stream(stream))
    _check(st, "nw_align_noalloc")


def align_noalloc_fits(m: int, n: int, score_only: bool = False) -> bool:
    st = lib().nw_align_noalloc_fits(int(m), int(n), SCORE_ONLY if score_only else 0)
    if st not in (NW_OK, -3):
        raise NWError(st, "nw_align_noalloc_fits")
    return st == NW_OK


def align_batch(pool: torch.Tensor, a_off: torch.Tensor, a_len: torch.Tensor, b_off: torch.Tensor,
                b_len: torch.Tensor, max_len: int, scoring=PAPER_SCORING, score_only: bool = False,
                path_off: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                stream=None):
    """Align many pairs from one pool.  Returns ``(scores, paths, path_off, path_len)``;
    the last three are None with ``score_only``.  When ``path_off`` is None it is
    the prefix sum of a_len + b_len."""
    npairs = int(a_len.numel())
    flags = SCORE_ONLY if score_only else 0
    dev = _dev()
    ws = _workspace(batch_workspace_size(npairs, max_len, flags), workspace)
    scores = torch.empty(npairs, dtype=torch.int32, device=dev)
    paths = plen = None
    if not score_only:
        caps = a_len.to(torch.int64) + b_len.to(torch.int64)
        if path_off is None:
            path_off = torch.zeros(npairs, dtype=torch.int64, device=dev)
            if npairs > 1:
                path_off[1:] = torch.cumsum(caps, 0)[:-1]
        total = int((path_off[-1] + caps[-1]).item()) if npairs else 1
        paths = torch.empty(max(total, 1), dtype=torch.uint8, device=dev)
        plen = torch.empty(npairs, dtype=torch.int32, device=dev)
    st = lib().nw_align_batch(npairs, _ptr(pool), _ptr(a_off), _ptr(a_len), _ptr(b_off), _ptr(b_len),
                              int(max_len), _sc(scoring), flags, _ptr(scores), _ptr(paths),
                              _ptr(path_off), _ptr(plen), _ptr(ws), ws.numel(), _stream(stream))
    _check(st, "nw_align_batch")
    return scores, paths, path_off, plen


def banded_workspace_size(npairs: int, max_len: int, flags: int = 0) -> int:
    out = _sz(0)
    _check(lib().nw_align_batch_banded_workspace_size(int(npairs), int(max_len), int(flags),
                                                      ctypes.byref(out)),
           "nw_align_batch_banded_workspace_size")
    return int(out.value)


def align_batch_banded(pool: torch.Tensor, a_off: torch.Tensor, a_len: torch.Tensor,
                       b_off: torch.Tensor, b_len: torch.Tensor, max_len: int,
                       scoring=PAPER_SCORING, w_init: torch.Tensor | None = None, w_default: int = 0,
                       fallback_frac: float = 0.5, score_only: bool = False,
                       path_off: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                       stream=None, doubling: bool = False, cells_score_only: torch.Tensor | None = None,
                       one_launch: bool = False):
    """Certified-band batch.  Returns ``(scores, paths, path_off, path_len, w_used, status,
    cells)`` (paths/path_off/path_len are None with ``score_only``).  ``doubling``
    widens a failed band by doubling (NW_BAND_DOUBLING); ``cells_score_only``
    (int64[npairs], optional) receives the cells swept score-only; ``one_launch``
    runs the score-only first passes inside the launch with paths
    (NW_BAND_ONE_LAUNCH: same results, slower)."""
    npairs = int(a_len.numel())
    flags = ((SCORE_ONLY if score_only else 0) | (BAND_DOUBLING if doubling else 0)
             | (BAND_ONE_LAUNCH if one_launch else 0))
    dev = _dev()
    ws = _workspace(banded_workspace_size(npairs, max_len, flags), workspace)
    scores = torch.empty(npairs, dtype=torch.int32, device=dev)
    w_used = torch.empty(npairs, dtype=torch.int32, device=dev)
    status = torch.empty(npairs, dtype=torch.uint8, device=dev)
    cells = torch.empty(npairs, dtype=torch.int64, device=dev)
    paths = plen = None
    if not score_only:
        caps = a_len.to(torch.int64) + b_len.to(torch.int64)
        if path_off is None:
            path_off = torch.zeros(npairs, dtype=torch.int64, device=dev)
            if npairs > 1:
                path_off[1:] = torch.cumsum(caps, 0)[:-1]
        total = int((path_off[-1] + caps[-1]).item()) if npairs else 1
        paths = torch.empty(max(total, 1), dtype=torch.uint8, device=dev)
        plen = torch.empty(npairs, dtype=torch.int32, device=dev)
    st = lib().nw_align_batch_banded(npairs, _ptr(pool), _ptr(a_off), _ptr(a_len), _ptr(b_off),
                                     _ptr(b_len), int(max_len), _sc(scoring), flags, _ptr(w_init),
                                     int(w_default), float(fallback_frac), _ptr(scores), _ptr(paths),
                                     _ptr(path_off), _ptr(plen), _ptr(w_used), _ptr(status),
                                     _ptr(cells), _ptr(cells_score_only), _ptr(ws), ws.numel(), _stream(stream))
    _check(st, "nw_align_batch_banded")
    return scores, paths, path_off, plen, w_used, status, cells


def _paths_out(a_len, b_len, npairs, path_off, dev):
    caps = a_len.to(torch.int64) + b_len.to(torch.int64)
    if path_off is None:
        path_off = torch.zeros(npairs, dtype=torch.int64, device=dev)
        if npairs > 1:
            path_off[1:] = torch.cumsum(caps, 0)[:-1]
    total = int((path_off[-1] + caps[-1]).item()) if npairs else 1
    paths = torch.empty(max(total, 1), dtype=torch.uint8, device=dev)
    plen = torch.empty(npairs, dtype=torch.int32, device=dev)
    return paths, path_off, plen


class Mlp:
    """Band-model state on the device: float32 master weights, their bfloat16
    copy (int16 bit patterns) and the Adam moments, wrapped in the library's
    ``nw_mlp`` struct."""

    def __init__(self, params):
        dev = _dev()
        p = torch.as_tensor(params, dtype=torch.float32).reshape(-1)
        if p.numel() != MLP_PARAMS:
            raise ValueError(f"expected {MLP_PARAMS} parameters, got {p.numel()}")
        self.params = p.to(dev).contiguous()
        self.params_bf16 = torch.empty(MLP_PARAMS, dtype=torch.int16, device=dev)
        self.adam_m = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=dev)
        self.adam_v = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=dev)
        self.state = MlpState(self.params.data_ptr(), self.params_bf16.data_ptr(),
                              self.adam_m.data_ptr(), self.adam_v.data_ptr(), 0)
        self.sync()

    @property
    def step(self) -> int:
        return int(self.state.step)

    def sync(self, stream=None):
        """Rewrite the bfloat16 copy from the master weights."""
        _check(lib().nw_mlp_sync(ctypes.byref(self.state), _stream(stream)), "nw_mlp_sync")


def mlp_features(pool, a_off, a_len, b_off, b_len, stream=None):
    """float32 [npairs, 259] feature rows (device)."""
    npairs = int(a_len.numel())
    x = torch.empty((npairs, MLP_INPUTS), dtype=torch.float32, device=_dev())
    _check(lib().nw_mlp_features(npairs, _ptr(pool), _ptr(a_off), _ptr(a_len), _ptr(b_off), _ptr(b_len),
                                 _ptr(x), _stream(stream)), "nw_mlp_features")
    return x


def mlp_forward(mlp: Mlp, x, stream=None):
    rows = int(x.shape[0])
    y = torch.empty(rows, dtype=torch.float32, device=_dev())
    _check(lib().nw_mlp_forward(ctypes.byref(mlp.state), rows, _ptr(x), _ptr(y), _stream(stream)),
           "nw_mlp_forward")
    return y


def mlp_widths(yhat, a_len, b_len, margin: float, stream=None):
    n = int(yhat.numel())
    w = torch.empty(n, dtype=torch.int32, device=_dev())
    _check(lib().nw_mlp_widths(n, _ptr(yhat), _ptr(a_len), _ptr(b_len), float(margin), _ptr(w),
                               _stream(stream)), "nw_mlp_widths")
    return w


def band_labels(scores, a_len, b_len, scoring=PAPER_SCORING, stream=None):
    """(w_cert int32, target float32 = log1p(w_cert)) device tensors."""
    n = int(scores.numel())
    dev = _dev()
    w = torch.empty(n, dtype=torch.int32, device=dev)
    t = torch.empty(n, dtype=torch.float32, device=dev)
    _check(lib().nw_band_labels(n, _ptr(scores), _ptr(a_len), _ptr(b_len), _sc(scoring), _ptr(w), _ptr(t),
                                _stream(stream)), "nw_band_labels")
    return w, t


def path_labels(paths, path_off, path_len, a_len, b_len, stream=None):
    """(w_path int32, target float32 = log1p(w_path)) device tensors from
    full-grid paths (as align_batch returns them)."""
    n = int(a_len.numel())
    dev = _dev()
    w = torch.empty(n, dtype=torch.int32, device=dev)
    t = torch.empty(n, dtype=torch.float32, device=dev)
    _check(lib().nw_path_labels(n, _ptr(paths), _ptr(path_off), _ptr(path_len), _ptr(a_len), _ptr(b_len),
                                _ptr(w), _ptr(t), _stream(stream)), "nw_path_labels")
    return w, t


def mlp_train_workspace_size(batch: int) -> int:
    out = _sz(0)
    _check(lib().nw_mlp_train_workspace_size(int(batch), ctypes.byref(out)), "nw_mlp_train_workspace_size")
    return int(out.value)


def mlp_train_step(mlp: Mlp, x, target, tau: float, lr: float, rows=None, want_grad: bool = False,
                   workspace=None, stream=None):
    """One step on rows (or all of x).  Returns (loss float32[1], grad float32[P] or None)."""
    batch = int(rows.numel()) if rows is not None else int(x.shape[0])
    dev = _dev()
    ws = _workspace(mlp_train_workspace_size(batch), workspace)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=dev) if want_grad else None
    _check(lib().nw_mlp_train_step(ctypes.byref(mlp.state), batch, _ptr(x), _ptr(target), _ptr(rows),
                                   float(tau), float(lr), _ptr(loss), _ptr(grad), _ptr(ws), ws.numel(),
                                   _stream(stream)), "nw_mlp_train_step")
    return loss, grad


def mlp_train_epoch(mlp: Mlp, x, target, order, batch: int, tau: float, lr: float, workspace=None,
                    stream=None):
    """One pass in the given order; returns the per-minibatch losses (device)."""
    n = int(order.numel())
    ws = _workspace(mlp_train_workspace_size(batch), workspace)
    losses = torch.empty(max((n + batch - 1) // batch, 1), dtype=torch.float32, device=_dev())
    _check(lib().nw_mlp_train_epoch(ctypes.byref(mlp.state), n, _ptr(x), _ptr(target), _ptr(order),
                                    int(batch), float(tau), float(lr), _ptr(losses), _ptr(ws), ws.numel(),
                                    _stream(stream)), "nw_mlp_train_epoch")
    return losses


def learned_workspace_size(npairs: int, max_len: int, flags: int = 0) -> int:
    out = _sz(0)
    _check(lib().nw_align_batch_learned_workspace_size(int(npairs), int(max_len), int(flags),
                                                       ctypes.byref(out)),
           "nw_align_batch_learned_workspace_size")
    return int(out.value)


def align_batch_learned(pool, a_off, a_len, b_off, b_len, max_len: int, mlp: Mlp, margin: float = 0.0,
                        scoring=PAPER_SCORING, fallback_frac: float = 0.5, score_only: bool = False,
                        path_off=None, workspace=None, stream=None, doubling: bool = False,
                        cells_score_only: torch.Tensor | None = None, one_launch: bool = False):
    """Learned-band batch; same returns and options as ``align_batch_banded``."""
    npairs = int(a_len.numel())
    flags = ((SCORE_ONLY if score_only else 0) | (BAND_DOUBLING if doubling else 0)
             | (BAND_ONE_LAUNCH if one_launch else 0))
    dev = _dev()
    ws = _workspace(learned_workspace_size(npairs, max_len, flags), workspace)
    scores = torch.empty(npairs, dtype=torch.int32, device=dev)
    w_used = torch.empty(npairs, dtype=torch.int32, device=dev)
    status = torch.empty(npairs, dtype=torch.uint8, device=dev)
    cells = torch.empty(npairs, dtype=torch.int64, device=dev)
    paths = plen = None
    if not score_only:
        paths, path_off, plen = _paths_out(a_len, b_len, npairs, path_off, dev)
    st = lib().nw_align_batch_learned(npairs, _ptr(pool), _ptr(a_off), _ptr(a_len), _ptr(b_off),
                                      _ptr(b_len), int(max_len), _sc(scoring), flags,
                                      ctypes.byref(mlp.state), float(margin), float(fallback_frac),
                                      _ptr(scores), _ptr(paths), _ptr(path_off), _ptr(plen),
                                      _ptr(w_used), _ptr(status), _ptr(cells), _ptr(cells_score_only), _ptr(ws),
                                      ws.numel(),
                                      _stream(stream))
    _check(st, "nw_align_batch_learned")
    return scores, paths, path_off, plen, w_used, status, cells


def autotune(pool, a_off, a_len, b_off, b_len, max_len: int, stream=None):
    """Measure the sweep-width costs on a sample batch (synchronises); returns
    the table {"dirs": [c128, c256, c512], "score": [...]}."""
    npairs = int(a_len.numel())
    dev = _dev()
    ws = _workspace(batch_workspace_size(npairs, max_len, 0), None)
    scores = torch.empty(npairs, dtype=torch.int32, device=dev)
    paths, path_off, plen = _paths_out(a_len, b_len, npairs, None, dev)
    costs = (ctypes.c_int32 * 6)()
    _check(lib().nw_autotune(npairs, _ptr(pool), _ptr(a_off), _ptr(a_len), _ptr(b_off), _ptr(b_len),
                             int(max_len), _ptr(scores), _ptr(paths), _ptr(path_off), _ptr(plen), _ptr(ws),
                             ws.numel(), costs, _stream(stream)), "nw_autotune")
    return {"dirs": list(costs[:3]), "score": list(costs[3:])}


def sweep_costs():
    """The current device's sweep-width cost table and whether it is tuned:
    ({"dirs": [c128, c256, c512], "score": [...]}, tuned)."""
    costs = (ctypes.c_int32 * 6)()
    tuned = ctypes.c_int32(0)
    _check(lib().nw_sweep_costs(costs, ctypes.byref(tuned)), "nw_sweep_costs")
    return {"dirs": list(costs[:3]), "score": list(costs[3:])}, bool(tuned.value)


def set_sweep_costs(table):
    """Install {"dirs": [...], "score": [...]} as the current device's table."""
    costs = (ctypes.c_int32 * 6)(*[int(x) for x in list(table["dirs"]) + list(table["score"])])
    _check(lib().nw_set_sweep_costs(costs), "nw_set_sweep_costs")


def autotune_cached(path, pool, a_off, a_len, b_off, b_len, max_len: int, config_class: str = "batch",
                    stream=None):
    """The autotuned cost table, kept in a JSON file under a key of (GPU
    architecture, compute-unit count, config class): installed from the file
    when the key is there, else measured with ``autotune`` on the given sample
    and added to the file.  Returns (table, measured)."""
    import json
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    key = f"{props.gcnArchName.split(':')[0]}|cu{props.multi_processor_count}|{config_class}"
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    if key in cache:
        set_sweep_costs(cache[key])
        return cache[key], False
    table = autotune(pool, a_off, a_len, b_off, b_len, max_len, stream)
    cache[key] = table
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return table, True


def center_star_workspace_size(nseq: int, max_len: int) -> int:
    out = _sz(0)
    _check(lib().nw_center_star_workspace_size(int(nseq), int(max_len), ctypes.byref(out)),
           "nw_center_star_workspace_size")
    return int(out.value)


def center_star(pool: torch.Tensor, off: torch.Tensor, lens: torch.Tensor, max_len: int,
                scores: torch.Tensor, scoring=PAPER_SCORING, gap_byte: int = 255, width_cap: int | None = None,
                workspace: torch.Tensor | None = None, stream=None):
    """Centre-star multiple alignment.  ``scores`` is the nseq x nseq matrix of
    ``allpairs``.  Returns ``(center, msa, width)`` device tensors: int32[1],
    uint8[nseq, width_cap] (row r = sequence r with gaps; the first ``width``
    bytes of each row are the alignment) and int64[1].  ``width_cap``
    defaults to the sum of the lengths, which always suffices."""
    nseq = int(lens.numel())
    dev = _dev()
    if width_cap is None:
        width_cap = max(int(lens.to(torch.int64).sum().item()), 1)
    ws = _workspace(center_star_workspace_size(nseq, max_len), workspace)
    center = torch.zeros(1, dtype=torch.int32, device=dev)
    width = torch.zeros(1, dtype=torch.int64, device=dev)
    msa = torch.empty((nseq, int(width_cap)), dtype=torch.uint8, device=dev)
    st = lib().nw_center_star(nseq, _ptr(pool), _ptr(off), _ptr(lens), int(max_len), _sc(scoring), _ptr(scores),
                              int(gap_byte), _ptr(center), _ptr(msa), int(width_cap), _ptr(width), _ptr(ws),
                              ws.numel(), _stream(stream))
    _check(st, "nw_center_star")
    return center, msa, width


def cooptimal_workspace_size(npairs: int, max_len: int, k: int = 0) -> int:
    out = _sz(0)
    _check(lib().nw_cooptimal_workspace_size(int(npairs), int(max_len), int(k), ctypes.byref(out)),
           "nw_cooptimal_workspace_size")
    return int(out.value)


def cooptimal(pool: torch.Tensor, a_off: torch.Tensor, a_len: torch.Tensor, b_off: torch.Tensor,
              b_len: torch.Tensor, max_len: int, scoring=PAPER_SCORING, k: int = 0,
              workspace: torch.Tensor | None = None, stream=None):
    """Co-optimal alignments of many pairs.  Returns ``(scores, counts, saturated)``
    (int32, int64 holding the count modulo 2^64 bit for bit, uint8) and, with
    ``k > 0``, also ``(paths, path_off, path_len, n_paths)``: pair q's path r
    is ``paths[path_off[q] + r*(a_len[q]+b_len[q]) :][:path_len[q, r]]``."""
    npairs = int(a_len.numel())
    dev = _dev()
    ws = _workspace(cooptimal_workspace_size(npairs, max_len, k), workspace)
    scores = torch.empty(npairs, dtype=torch.int32, device=dev)
    counts = torch.empty(npairs, dtype=torch.int64, device=dev)
    sat = torch.empty(npairs, dtype=torch.uint8, device=dev)
    paths = path_off = path_len = n_paths = None
    if k > 0:
        caps = (a_len.to(torch.int64) + b_len.to(torch.int64)) * k
        path_off = torch.cumsum(caps, 0) - caps
        paths = torch.empty(max(int(caps.sum().item()), 1), dtype=torch.uint8, device=dev)
        path_len = torch.zeros((npairs, k), dtype=torch.int32, device=dev)
        n_paths = torch.empty(npairs, dtype=torch.int32, device=dev)
    st = lib().nw_cooptimal(npairs, _ptr(pool), _ptr(a_off), _ptr(a_len), _ptr(b_off), _ptr(b_len), int(max_len),
                            _sc(scoring), _ptr(scores), _ptr(counts), _ptr(sat), int(k), _ptr(paths),
                            _ptr(path_off), _ptr(path_len), _ptr(n_paths), _ptr(ws), ws.numel(), _stream(stream))
    _check(st, "nw_cooptimal")
    if k > 0:
        return scores, counts, sat, paths, path_off, path_len, n_paths
    return scores, counts, sat


def allpairs(pool: torch.Tensor, off: torch.Tensor, lens: torch.Tensor, max_len: int,
             scoring=PAPER_SCORING, workspace: torch.Tensor | None = None, stream=None):
    """nseq x nseq int32 score matrix (device)."""
    nseq = int(lens.numel())
    dev = _dev()
    ws = _workspace(allpairs_workspace_size(nseq, max_len), workspace)
    out = torch.empty((nseq, nseq), dtype=torch.int32, device=dev)
    st = lib().nw_allpairs_scores(nseq, _ptr(pool), _ptr(off), _ptr(lens), int(max_len), _sc(scoring),
                                  _ptr(out), _ptr(ws), ws.numel(), _stream(stream))
    _check(st, "nw_allpairs_scores")
    return out


def init():
    """nw_init: one-time set-up of the library on the current device."""
    _check(lib().nw_init(), "nw_init")


def sync(stream=None):
    """nw_sync: synchronise the stream, then raise NWError(NW_EDEVICE) if the
    kernels reported a device fault."""
    _check(lib().nw_sync(_stream(stream)), "nw_sync")


def set_wait_limit(polls: int):
    """nw_set_wait_limit: polls a bounded wait between waves makes before it
    gives up (0 restores the default).  A testing hook for the fault path."""
    _check(lib().nw_set_wait_limit(int(polls)), "nw_set_wait_limit")


def set_walk_limit(moves: int):
    """nw_set_walk_limit: nw_align (from 512 columns) walks paths of at most
    `moves` moves back with one wave and longer ones strip-parallel (0
    restores the default, 1 sends every such pair to the parallel walk)."""
    _check(lib().nw_set_walk_limit(int(moves)), "nw_set_walk_limit")


def profile_begin():
    """Start recording HIP events around every library kernel launch."""
    _check(lib().nw_profile_begin(), "nw_profile_begin")


def profile_end():
    """Stop recording; call after synchronising.  Returns {kernel: (launches, total_ms)}."""
    cap = 64
    buf = (KernelTime * cap)()
    cnt = _i32(0)
    _check(lib().nw_profile_end(buf, cap, ctypes.byref(cnt)), "nw_profile_end")
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms))
            for i in range(min(cnt.value, cap))}
