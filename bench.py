#!/usr/bin/env python3
"""Benchmark of the Needleman-Wunsch hot path on one MI355X.

Workload: the single long pair -- a 65,536-base random ancestor and its
10%-mutated descendant (70% substitutions, 15% insertions, 15% deletions,
indel lengths geometric(0.5)), seeded; paper scoring +1/-1/-1; full int32
DP with 2-bit directions and the tie-break traceback.  One step = one
nw_align call (fill + traceback) on inputs already resident in HBM.

Prints one JSON line: GCUPS (m*n cell updates per second), the fill
kernel's roofline position (live HIP-event timing of the fill launches in
the timed region), and the CPU oracle's rate on the same pair.

The same line carries the learned-band batch beside plain full-DP batching
(`learned_band`): 8192 pairs of lengths 1,000..20,000 at divergence 1..30%,
the band model trained on 4096 pairs from disjoint seeds (labels from the
full-DP method), then full-DP and learned-band runs of the whole batch with
paths, compared for identical scores and paths on the device.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT32_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # CUs * SIMDs * lanes * clock: 39.32 T lane-ops/s
FILL_OPS_PER_CELL = 5  # diagonal term, vertical add, max3, tag clear, tag shift
# counting optimal paths: diagonal term, max, three equality tests, six 32-bit selects, two 64-bit adds
COUNT_OPS_PER_CELL = 13
KERNEL_SOURCES = ["paper_2412_21103_amd/csrc/nw_common.h", "paper_2412_21103_amd/csrc/nw_strip.h",
                  "paper_2412_21103_amd/csrc/nw_single.hip"]
COUNTERS = os.path.join(ROOT, "profiles", "fill_coop_long_pair_65536.counters.json")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_record():
    """HBM bytes per fill launch from the committed rocprofv3 counter summary,
    or None if the kernel sources changed since the counters were taken."""
    if not os.path.exists(COUNTERS):
        return None
    rec = json.load(open(COUNTERS))
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def learned_band(npairs: int, warmup: int, dev, reps: int = 3):
    """Full-DP batch vs learned certified band on the learned-band workload."""
    import numpy as np
    import torch

    import paper_2412_21103_amd as nwp
    from paper_2412_21103_amd import band_model
    from workloads import config_band_batch, pack_pairs

    def to_dev(pairs):
        pool, ao, al, bo, bl = pack_pairs(pairs)
        t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to(dev)
        return (t(pool, np.uint8), t(ao, np.int64), t(al, np.int32), t(bo, np.int64), t(bl, np.int32),
                int(max(al.max(), bl.max())))

    print(f"bench: learned band, generating {npairs} + {npairs // 2} pairs", file=sys.stderr, flush=True)
    test = to_dev(config_band_batch(npairs=npairs))
    train = to_dev(config_band_batch(seed=5100, npairs=max(npairs // 2, 1)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, _, _, target = band_model.features_and_labels(*train)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mlp, hist = band_model.train(x, target, epochs=200, batch=256, lr=3e-3, tau=0.9, seed=1)
    t2 = time.perf_counter()
    print(f"bench: labels {t1 - t0:.2f} s, training {t2 - t1:.2f} s, loss {hist[0]:.3f} -> {hist[-1]:.4f}",
          file=sys.stderr, flush=True)
    del train, x, target
    cells = float((test[2].to(torch.float64) * test[4].to(torch.float64)).sum())
    ws = torch.empty(nwp.learned_workspace_size(npairs, test[5]), dtype=torch.uint8, device=dev)
    margin = 0.1

    def run(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) / reps

    print("bench: full-DP batch", file=sys.stderr, flush=True)
    ref, t_full = run(lambda: nwp.align_batch(*test, workspace=ws))
    s_ref, p_ref, poff, plen_ref = ref
    print("bench: learned-band batch", file=sys.stderr, flush=True)
    out, t_band = run(lambda: nwp.align_batch_learned(*test, mlp, margin, path_off=poff, workspace=ws))
    s, p, _, plen, w_used, status, swept = out
    # identical scores, lengths and every path byte (compared on the device)
    plen64 = plen_ref.to(torch.int64)
    starts = torch.repeat_interleave(poff, plen64)
    base = torch.repeat_interleave(torch.cumsum(plen64, 0) - plen64, plen64)
    idx = starts + torch.arange(int(plen64.sum()), device=dev) - base
    exact = bool(torch.equal(s, s_ref) and torch.equal(plen, plen_ref) and torch.equal(p[idx], p_ref[idx]))
    st = status.cpu().numpy()
    return {"workload": f"band_batch_{npairs}", "pairs": npairs, "full_equivalent_cells": cells,
            "full_dp_gcups": round(cells / t_full / 1e9, 1), "full_dp_ms": round(t_full * 1e3, 2),
            "learned_effective_gcups": round(cells / t_band / 1e9, 1),
            "learned_computed_gcups": round(float(swept.sum()) / t_band / 1e9, 1),
            "learned_ms": round(t_band * 1e3, 2), "speedup_vs_full_dp": round(t_full / t_band, 3),
            "cells_swept_frac": round(float(swept.sum()) / cells, 4),
            "certified_first_pass": round(float(np.mean(st & 1)), 4),
            "full_grid_frac": round(float(np.mean((st & 0x40) != 0)), 4), "margin": margin,
            "train_pairs": max(npairs // 2, 1), "train_s": round(t2 - t1, 3), "label_dp_s": round(t1 - t0, 3),
            "bit_exact_vs_full_dp": exact}


def common_fields(args, value, ms_per_step, config, roofline, cpu, metric_suffix=""):
    return {
        "metric": "GCUPS (cell updates/s) full-DP and certified learned-band, 1 MI355X, bit-exact"
                  + metric_suffix,
        "value": round(value, 3),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": config,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }


def alu_roofline(kernel, cells, kernel_ms, ops_per_cell):
    if not kernel_ms:
        return None
    achieved = ops_per_cell * cells / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_INT32_TOPS, 3),
            "unit": "T int32 lane-ops/s", "frac": round(achieved / PEAK_INT32_TOPS, 4), "traffic": None,
            "kernel": kernel, "kernel_ms": round(kernel_ms, 4), "ops_per_cell": ops_per_cell}


def timed_steps(step, args, sync):
    for _ in range(args.warmup):
        step()
    sync()
    import paper_2412_21103_amd as nwp
    print(f"bench: timing {args.steps} steps", file=sys.stderr, flush=True)
    nwp.profile_begin()
    sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    sync()
    t1 = time.perf_counter()
    return (t1 - t0) * 1e3 / args.steps, nwp.profile_end()


def bench_batch(args):
    """4096 pairs, m in [100, 2000], 5-15% mutated, scores + paths, one launch per step."""
    import ctypes

    import numpy as np
    import torch

    import paper_2412_21103_amd as nwp
    from workloads import config_batch, pack_pairs

    print("bench: generating the 4096-pair batch", file=sys.stderr, flush=True)
    pairs = config_batch()
    pool, ao, al, bo, bl = pack_pairs(pairs)
    npairs = len(pairs)
    max_len = int(max(al.max(), bl.max()))
    cells = int((al.astype(np.int64) * bl.astype(np.int64)).sum())
    caps = al.astype(np.int64) + bl.astype(np.int64)
    poff = np.concatenate([[0], np.cumsum(caps)[:-1]]).astype(np.int64)
    dev = torch.device("cuda", 0)
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to(dev)
    d = [t(pool, np.uint8), t(ao, np.int64), t(al, np.int32), t(bo, np.int64), t(bl, np.int32)]
    d_poff = t(poff, np.int64)
    scores = torch.empty(npairs, dtype=torch.int32, device=dev)
    paths = torch.empty(int(caps.sum()), dtype=torch.uint8, device=dev)
    plen = torch.empty(npairs, dtype=torch.int32, device=dev)
    ws_bytes = nwp.batch_workspace_size(npairs, max_len, 0)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    L = nwp.lib()
    sc = nwp.Scoring(*nwp.PAPER_SCORING)
    stream = torch.cuda.current_stream()
    vp = ctypes.c_void_p
    ptr = lambda x: vp(x.data_ptr())

    def step():
        st = L.nw_align_batch(npairs, *[ptr(x) for x in d], max_len, sc, 0, ptr(scores), ptr(paths),
                              ptr(d_poff), ptr(plen), ptr(ws), ws_bytes, vp(stream.cuda_stream))
        if st != 0:
            raise nwp.NWError(st, "nw_align_batch")

    ms, prof = timed_steps(step, args, torch.cuda.synchronize)
    k = prof.get("nw_batch")
    roof = alu_roofline("nw_batch", cells, k[1] / k[0] if k else None, FILL_OPS_PER_CELL)
    cpu = exact = None
    if not args.no_cpu_baseline:
        import oracle
        nt = oracle.max_threads()
        print(f"bench: CPU oracle on the whole batch ({nt} threads)", file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        s_ref, p_ref = oracle.align_batch(pool, ao, al, bo, bl, oracle.PAPER_SCORING)
        c1 = time.perf_counter()
        s_gpu = scores.cpu().numpy()
        pg, pl = paths.cpu().numpy(), plen.cpu().numpy()
        exact = bool((s_gpu == s_ref).all() and all(
            np.array_equal(pg[poff[i]:poff[i] + pl[i]], p_ref[i]) for i in range(npairs)))
        cpu = {"value": round(cells / (c1 - c0) / 1e9, 4), "unit": "GCUPS", "cores": nt, "kind": "oracle",
               "sample": f"the whole batch ({cells} cells), scores + paths, full int32 matrix per pair, "
                         f"OpenMP over pairs, {round(c1 - c0, 2)} s"}
    config = {"workload": f"batch_{npairs}", "pairs": npairs, "cells": cells, "max_len": max_len,
              "scoring": list(nwp.PAPER_SCORING), "traceback": True, "bit_exact_vs_oracle": exact}
    return common_fields(args, cells / (ms * 1e-3) / 1e9, ms, config, roof, cpu)


def bench_allpairs(args):
    """All-pairs score matrix of 512 sequences (lengths 500..5000), score-only."""
    import ctypes

    import numpy as np
    import torch

    import paper_2412_21103_amd as nwp
    from workloads import config_allpairs, pack_seqs

    print("bench: generating the 512 sequences", file=sys.stderr, flush=True)
    seqs = config_allpairs()
    pool, off, lens = pack_seqs(seqs)
    nseq = len(seqs)
    max_len = int(lens.max())
    l64 = lens.astype(np.int64)
    cells = int((l64.sum() ** 2 - (l64 ** 2).sum()) // 2)  # i < j pairs
    dev = torch.device("cuda", 0)
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to(dev)
    d = [t(pool, np.uint8), t(off, np.int64), t(lens, np.int32)]
    out = torch.empty((nseq, nseq), dtype=torch.int32, device=dev)
    ws_bytes = nwp.allpairs_workspace_size(nseq, max_len)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    L = nwp.lib()
    sc = nwp.Scoring(*nwp.PAPER_SCORING)
    stream = torch.cuda.current_stream()
    vp = ctypes.c_void_p
    ptr = lambda x: vp(x.data_ptr())

    def step():
        st = L.nw_allpairs_scores(nseq, *[ptr(x) for x in d], max_len, sc, ptr(out), ptr(ws), ws_bytes,
                                  vp(stream.cuda_stream))
        if st != 0:
            raise nwp.NWError(st, "nw_allpairs_scores")

    ms, prof = timed_steps(step, args, torch.cuda.synchronize)
    k = prof.get("nw_allpairs")
    roof = alu_roofline("nw_allpairs", cells, k[1] / k[0] if k else None, 2)
    cpu = exact = None
    if not args.no_cpu_baseline:
        import oracle
        nt = oracle.max_threads()
        ns = 64
        sub = seqs[:ns]
        sp, so, sl = pack_seqs(sub)
        s64 = sl.astype(np.int64)
        sub_cells = int((s64.sum() ** 2 - (s64 ** 2).sum()) // 2)
        print(f"bench: CPU oracle on the first {ns} sequences ({nt} threads)", file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        M = oracle.allpairs(sp, so, sl, oracle.PAPER_SCORING)
        c1 = time.perf_counter()
        exact = bool(np.array_equal(out.cpu().numpy()[:ns, :ns], M))
        cpu = {"value": round(sub_cells / (c1 - c0) / 1e9, 4), "unit": "GCUPS", "cores": nt, "kind": "oracle",
               "sample": f"the first {ns} sequences ({ns * (ns - 1) // 2} pairs, {sub_cells} cells), "
                         f"score-only, OpenMP over pairs, {round(c1 - c0, 2)} s"}
    config = {"workload": f"allpairs_{nseq}", "sequences": nseq, "pairs": nseq * (nseq - 1) // 2,
              "cells": cells, "scoring": list(nwp.PAPER_SCORING), "traceback": False,
              "bit_exact_vs_oracle_sample": exact}
    return common_fields(args, cells / (ms * 1e-3) / 1e9, ms, config, roof, cpu)


def bench_cooptimal(args):
    """Co-optimal alignments of the 4096-pair batch: the number of optimal
    paths of every pair per step (counts only), and beside it the first four
    paths of every pair."""
    import ctypes

    import numpy as np
    import torch

    import paper_2412_21103_amd as nwp
    from workloads import config_batch, pack_pairs

    print("bench: generating the 4096-pair batch", file=sys.stderr, flush=True)
    pairs = config_batch()
    pool, ao, al, bo, bl = pack_pairs(pairs)
    npairs = len(pairs)
    max_len = int(max(al.max(), bl.max()))
    cells = int((al.astype(np.int64) * bl.astype(np.int64)).sum())
    dev = torch.device("cuda", 0)
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to(dev)
    d = [t(pool, np.uint8), t(ao, np.int64), t(al, np.int32), t(bo, np.int64), t(bl, np.int32)]
    scores = torch.empty(npairs, dtype=torch.int32, device=dev)
    counts = torch.empty(npairs, dtype=torch.int64, device=dev)
    sat = torch.empty(npairs, dtype=torch.uint8, device=dev)
    ws_bytes = nwp.cooptimal_workspace_size(npairs, max_len, 0)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    L = nwp.lib()
    sc = nwp.Scoring(*nwp.PAPER_SCORING)
    stream = torch.cuda.current_stream()
    vp = ctypes.c_void_p
    ptr = lambda x: vp(x.data_ptr())
    null = vp(0)

    def step():
        st = L.nw_cooptimal(npairs, *[ptr(x) for x in d], max_len, sc, ptr(scores), ptr(counts), ptr(sat), 0,
                            null, null, null, null, ptr(ws), ws_bytes, vp(stream.cuda_stream))
        if st != 0:
            raise nwp.NWError(st, "nw_cooptimal")

    ms, prof = timed_steps(step, args, torch.cuda.synchronize)
    k = prof.get("nw_cooptimal")
    roof = alu_roofline("nw_cooptimal", cells, k[1] / k[0] if k else None, COUNT_OPS_PER_CELL)
    # the first four paths of every pair, same pairs
    kp = 4
    print(f"bench: counts + first {kp} paths", file=sys.stderr, flush=True)
    wsk = torch.empty(nwp.cooptimal_workspace_size(npairs, max_len, kp), dtype=torch.uint8, device=dev)
    out = nwp.cooptimal(*d, max_len, nwp.PAPER_SCORING, k=kp, workspace=wsk)
    torch.cuda.synchronize()
    nwp.profile_begin()
    for _ in range(2):
        out = nwp.cooptimal(*d, max_len, nwp.PAPER_SCORING, k=kp, workspace=wsk)
    torch.cuda.synchronize()
    kprof = nwp.profile_end().get("nw_cooptimal_paths")
    paths_ms = round(kprof[1] / kprof[0], 4) if kprof else None
    npaths = out[6].cpu().numpy()
    same = bool(torch.equal(out[0], scores) and torch.equal(out[1], counts) and torch.equal(out[2], sat))
    c_gpu = counts.cpu().numpy().view(np.uint64)
    cpu = exact = None
    if not args.no_cpu_baseline:
        import oracle
        from oracle import coopt
        nt = oracle.max_threads()
        print(f"bench: CPU oracle counts on the whole batch ({nt} threads)", file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        s_ref, n_ref, f_ref = coopt.count_batch(pool, ao, al, bo, bl, oracle.PAPER_SCORING)
        c1 = time.perf_counter()
        exact = bool(np.array_equal(scores.cpu().numpy(), s_ref) and np.array_equal(c_gpu, n_ref)
                     and np.array_equal(sat.cpu().numpy(), f_ref))
        cpu = {"value": round(cells / (c1 - c0) / 1e9, 4), "unit": "GCUPS", "cores": nt, "kind": "oracle",
               "sample": f"the whole batch ({cells} cells), scores + counts mod 2^64 + flags, two rows per pair, "
                         f"OpenMP over pairs, {round(c1 - c0, 2)} s"}
    config = {"workload": f"cooptimal_batch_{npairs}", "pairs": npairs, "cells": cells, "max_len": max_len,
              "scoring": list(nwp.PAPER_SCORING), "counts_only": True,
              "pairs_with_one_optimal_path": int((c_gpu == 1).sum()),
              "median_count": float(np.median(c_gpu.astype(np.float64))),
              "saturated_pairs": int(sat.sum().item()),
              "first_paths_k": kp, "first_paths_kernel_ms": paths_ms,
              "first_paths_listed": int(npaths.sum()),
              "first_paths_counts_equal": same, "bit_exact_vs_oracle": exact}
    return common_fields(args, cells / (ms * 1e-3) / 1e9, ms, config, roof, cpu)


def bench_center_star(args):
    """Centre-star multiple alignment of the 512 all-pairs sequences: the
    all-pairs score matrix, then the centre pick, the 511 alignments to the
    centre with traceback and the merge, one pass per step."""
    import ctypes

    import numpy as np
    import torch

    import paper_2412_21103_amd as nwp
    from workloads import config_allpairs, pack_seqs

    print("bench: generating the 512 sequences", file=sys.stderr, flush=True)
    seqs = config_allpairs()
    pool, off, lens = pack_seqs(seqs)
    nseq = len(seqs)
    max_len = int(lens.max())
    l64 = lens.astype(np.int64)
    cells_all = int((l64.sum() ** 2 - (l64 ** 2).sum()) // 2)
    width_cap = int(l64.sum())
    dev = torch.device("cuda", 0)
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to(dev)
    d = [t(pool, np.uint8), t(off, np.int64), t(lens, np.int32)]
    S = torch.empty((nseq, nseq), dtype=torch.int32, device=dev)
    center = torch.zeros(1, dtype=torch.int32, device=dev)
    width = torch.zeros(1, dtype=torch.int64, device=dev)
    msa = torch.empty((nseq, width_cap), dtype=torch.uint8, device=dev)
    ws_a = nwp.allpairs_workspace_size(nseq, max_len)
    ws_c = nwp.center_star_workspace_size(nseq, max_len)
    ws = torch.empty(max(ws_a, ws_c), dtype=torch.uint8, device=dev)
    L = nwp.lib()
    sc = nwp.Scoring(*nwp.PAPER_SCORING)
    stream = torch.cuda.current_stream()
    vp = ctypes.c_void_p
    ptr = lambda x: vp(x.data_ptr())

    def step():
        st = L.nw_allpairs_scores(nseq, *[ptr(x) for x in d], max_len, sc, ptr(S), ptr(ws), ws_a,
                                  vp(stream.cuda_stream))
        if st != 0:
            raise nwp.NWError(st, "nw_allpairs_scores")
        st = L.nw_center_star(nseq, *[ptr(x) for x in d], max_len, sc, ptr(S), 255, ptr(center), ptr(msa),
                              width_cap, ptr(width), ptr(ws), ws_c, vp(stream.cuda_stream))
        if st != 0:
            raise nwp.NWError(st, "nw_center_star")

    ms, prof = timed_steps(step, args, torch.cuda.synchronize)
    c = int(center.item())
    w = int(width.item())
    cells_star = int(l64[c] * (l64.sum() - l64[c]))
    cells = cells_all + cells_star
    k = prof.get("nw_allpairs")
    roof = alu_roofline("nw_allpairs", cells_all, k[1] / k[0] if k else None, 2)
    phases = {name: round(v[1] / v[0], 4) for name, v in prof.items()
              if name in ("nw_allpairs", "nw_msa_center", "nw_batch", "nw_msa_merge") and v[0]}
    cpu = exact = None
    if not args.no_cpu_baseline:
        import oracle
        from oracle import msa as omsa
        nt = oracle.max_threads()
        ns = 48
        sub = seqs[:ns]
        sp, so, sl = pack_seqs(sub)
        s64 = sl.astype(np.int64)
        print(f"bench: CPU oracle centre star on the first {ns} sequences ({nt} threads)", file=sys.stderr,
              flush=True)
        c0 = time.perf_counter()
        M_ref = oracle.allpairs(sp, so, sl, oracle.PAPER_SCORING)
        c_ref, A_ref = omsa.center_star(sub, oracle.PAPER_SCORING, 255, scores=M_ref)
        c1 = time.perf_counter()
        sub_cells = int((s64.sum() ** 2 - (s64 ** 2).sum()) // 2 + s64[c_ref] * (s64.sum() - s64[c_ref]))
        gd = [t(sp, np.uint8), t(so, np.int64), t(sl, np.int32)]
        gS = nwp.allpairs(*gd, int(sl.max()), nwp.PAPER_SCORING)
        gc, gM, gw = nwp.center_star(*gd, int(sl.max()), gS, nwp.PAPER_SCORING, gap_byte=255)
        gw = int(gw.item())
        exact = bool(int(gc.item()) == c_ref and gw == A_ref.shape[1]
                     and np.array_equal(gM.cpu().numpy()[:, :gw], A_ref)
                     and np.array_equal(gS.cpu().numpy(), M_ref))
        cpu = {"value": round(sub_cells / (c1 - c0) / 1e9, 4), "unit": "GCUPS", "cores": nt, "kind": "oracle",
               "sample": f"the first {ns} sequences ({sub_cells} cells): all-pairs scores (OpenMP over pairs), "
                         f"the {ns - 1} alignments to the centre and the merge (one thread), "
                         f"{round(c1 - c0, 2)} s"}
    config = {"workload": f"center_star_{nseq}", "sequences": nseq, "cells": cells, "allpairs_cells": cells_all,
              "alignment_cells": cells_star, "center": c, "width": w, "scoring": list(nwp.PAPER_SCORING),
              "phase_ms": phases, "bit_exact_vs_oracle_sample": exact}
    return common_fields(args, cells / (ms * 1e-3) / 1e9, ms, config, roof, cpu)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=["long_pair", "batch", "allpairs", "center_star", "cooptimal"], default="long_pair")
    ap.add_argument("--length", type=int, default=65536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-band", action="store_true", help="skip the learned-band batch")
    ap.add_argument("--band-pairs", type=int, default=8192)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="first run a plain device copy of BYTES bytes (int32 elementwise), the reference "
                         "kernel that scales the HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(pairs are independent; several GPUs would each run a cost-balanced share of them)", file=sys.stderr)
        return 2
    if args.copy_probe > 0:
        import torch
        src = torch.ones(args.copy_probe // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            torch.mul(src, 1, out=dst)
        torch.cuda.synchronize()
        print(f"bench: copy probe of {args.copy_probe} bytes done", file=sys.stderr, flush=True)
        del src, dst
    if args.workload == "batch":
        print(json.dumps(bench_batch(args)), flush=True)
        return 0
    if args.workload == "allpairs":
        print(json.dumps(bench_allpairs(args)), flush=True)
        return 0
    if args.workload == "center_star":
        print(json.dumps(bench_center_star(args)), flush=True)
        return 0
    if args.workload == "cooptimal":
        print(json.dumps(bench_cooptimal(args)), flush=True)
        return 0

    import ctypes

    import numpy as np
    import torch

    import paper_2412_21103_amd as nwp
    from workloads import config_long_pair

    print(f"bench: generating the {args.length}-base pair", file=sys.stderr, flush=True)
    pair = config_long_pair(length=args.length)
    a, b = pair.a[0], pair.b[0]
    m, n = int(a.shape[0]), int(b.shape[0])
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(0)
    da = torch.from_numpy(a).to(dev)
    db = torch.from_numpy(b).to(dev)
    ws_bytes = nwp.align_workspace_size(m, n, 0)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    score = torch.empty(1, dtype=torch.int32, device=dev)
    path = torch.empty(m + n, dtype=torch.uint8, device=dev)
    plen = torch.empty(1, dtype=torch.int64, device=dev)
    L = nwp.lib()
    sc = nwp.Scoring(*nwp.PAPER_SCORING)
    stream = torch.cuda.current_stream()
    vp = ctypes.c_void_p

    def step():
        st = L.nw_align(vp(da.data_ptr()), m, vp(db.data_ptr()), n, sc, 0, vp(score.data_ptr()),
                        vp(path.data_ptr()), m + n, vp(plen.data_ptr()), vp(ws.data_ptr()), ws_bytes,
                        vp(stream.cuda_stream))
        if st != 0:
            raise nwp.NWError(st, "nw_align")

    print(f"bench: {m} x {n}, warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"bench: timing {args.steps} steps", file=sys.stderr, flush=True)
    nwp.profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = nwp.profile_end()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    cells = m * n
    gcups = cells / (ms_per_step * 1e-3) / 1e9

    gpu_score = int(score.item())
    k = int(plen.item())
    gpu_path = path[:k].cpu().numpy()

    fill = prof.get("nw_fill_coop")
    fill_ms = fill[1] / fill[0] if fill else None
    tb = [prof[k] for k in ("nw_tb_spec", "nw_tb_fix", "nw_tb_emit") if k in prof]
    walk_ms = sum(v[1] / v[0] for v in tb) if tb else None
    roofline = None
    if fill_ms:
        achieved = FILL_OPS_PER_CELL * cells / (fill_ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_INT32_TOPS, 3),
                    "unit": "T int32 lane-ops/s", "frac": round(achieved / PEAK_INT32_TOPS, 4),
                    "traffic": traffic_record(), "kernel": "nw_fill_coop",
                    "kernel_ms": round(fill_ms, 4), "ops_per_cell": FILL_OPS_PER_CELL}

    cpu = None
    exact = None
    if not args.no_cpu_baseline:
        import oracle
        print("bench: CPU oracle on the same pair (one thread)", file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        s_ref, p_ref = oracle.align(a, b, oracle.PAPER_SCORING, full_limit_bytes=0)
        c1 = time.perf_counter()
        exact = bool(s_ref == gpu_score and np.array_equal(p_ref, gpu_path))
        cpu = {"value": round(cells / (c1 - c0) / 1e9, 4), "unit": "GCUPS", "cores": 1,
               "kind": "oracle",
               "sample": f"the whole {m} x {n} pair, score + traceback, two score rows + "
                         f"a direction byte per cell, {round(c1 - c0, 2)} s"}

    band = None if args.no_band else learned_band(args.band_pairs, args.warmup, dev)

    out = {
        "metric": "GCUPS (cell updates/s) full-DP and certified learned-band, 1 MI355X, bit-exact",
        "value": round(gcups, 3),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"long_pair_{args.length}", "m": m, "n": n, "mutation_rate": 0.10,
                   "scoring": list(nwp.PAPER_SCORING), "traceback": True,
                   "fill_ms": round(fill_ms, 4) if fill_ms else None,
                   "traceback_ms": round(walk_ms, 4) if walk_ms else None,
                   "bit_exact_vs_oracle": exact},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "learned_band": band,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
