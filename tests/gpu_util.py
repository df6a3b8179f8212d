"""Helpers for the GPU parity tests: move numpy inputs to the device, call the
library through its binding, bring results back."""
import sys

import numpy as np
import torch

import paper_2412_21103_amd as nwp


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_u8(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.uint8)).to("cuda")


def gpu_align(a, b, scoring=(1, -1, -1), score_only=False):
    da, db = dev_u8(a), dev_u8(b)
    s, p, pl = nwp.align(da, db, scoring, score_only=score_only)
    torch.cuda.synchronize()
    score = int(s.item())
    if score_only:
        return score, None
    k = int(pl.item())
    return score, p[:k].cpu().numpy() if k > 0 else np.zeros(0, np.uint8)


def gpu_batch(pool, a_off, a_len, b_off, b_len, max_len, scoring=(1, -1, -1), score_only=False):
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")
    s, paths, poff, plen = nwp.align_batch(dev_u8(pool), t(a_off, np.int64), t(a_len, np.int32),
                                           t(b_off, np.int64), t(b_len, np.int32), max_len, scoring,
                                           score_only=score_only)
    torch.cuda.synchronize()
    scores = s.cpu().numpy()
    if score_only:
        return scores, None
    paths = paths.cpu().numpy()
    poff = poff.cpu().numpy()
    plen = plen.cpu().numpy()
    return scores, [paths[poff[k]:poff[k] + max(plen[k], 0)] for k in range(len(plen))], plen


def gpu_allpairs(pool, off, lens, max_len, scoring=(1, -1, -1)):
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to("cuda")
    M = nwp.allpairs(dev_u8(pool), t(off, np.int64), t(lens, np.int32), max_len, scoring)
    torch.cuda.synchronize()
    return M.cpu().numpy()
