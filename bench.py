#!/usr/bin/env python3
"""Benchmark of the Needleman-Wunsch hot path on one MI355X.

Default workload (the metric's configuration): the learned-band batch --
8192 pairs of lengths 1,000..20,000 at divergence 1..30% and indel fraction
5..50%, seeded; paper scoring +1/-1/-1; scores and tie-break paths.  One step
is one nw_align_batch_learned call (k-mer features, network, half-widths,
certified banded fill, widening a failed band to the width its score
certifies, traceback) on inputs already resident in HBM.  The band model is
trained in the same run on 4096 pairs from disjoint seeds, on the excursion
of the full-DP method's own paths beyond the straight band.  Beside it on
the same GPU and inputs: full DP (nw_align_batch); the certified band from
the best constant starting half-width (the method without the network,
chosen on the training pairs by wall time); and both again under the
doubling rule (the network then trained on the certified width).  Every
score and path byte is compared with full DP on the device, and the CPU
oracle runs on a bounded sample of the pairs.

Prints one JSON line: effective GCUPS of the learned band (full-equivalent
m*n cells per second of wall time) as `value`, the banded kernel's roofline
position (HIP-event timing of its launches in the timed region), and the
oracle's rate.  Extra keys carry the single long pair (65,536 bases) and the
single 1024-base pair.  Other workloads: --workload long_pair | single |
batch | allpairs | center_star | cooptimal.
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
SCORE_OPS_PER_CELL = 2  # score only: diagonal term, max3
# counting optimal paths: diagonal term, max, three equality tests, six 32-bit selects, two 64-bit adds
COUNT_OPS_PER_CELL = 13
COOP_SOURCES = ["paper_2412_21103_amd/csrc/nw_common.h", "paper_2412_21103_amd/csrc/nw_strip.h",
                "paper_2412_21103_amd/csrc/nw_single.hip"]
BAND_SOURCES = ["paper_2412_21103_amd/csrc/nw_common.h", "paper_2412_21103_amd/csrc/nw_strip.h",
                "paper_2412_21103_amd/csrc/nw_batch.hip"]
COOP_COUNTERS = os.path.join(ROOT, "profiles", "fill_coop_long_pair_65536.counters.json")
BAND_COUNTERS = os.path.join(ROOT, "profiles", "batch_banded_band_batch_8192.counters.json")
BAND_VALU = os.path.join(ROOT, "profiles", "batch_banded_band_batch_8192.valu.json")
BATCH_COUNTERS = os.path.join(ROOT, "profiles", "batch_batch_4096.counters.json")
BATCH_VALU = os.path.join(ROOT, "profiles", "batch_batch_4096.valu.json")
COOP_VALU = os.path.join(ROOT, "profiles", "fill_coop_long_pair_65536.valu.json")
ALLPAIRS_VALU = os.path.join(ROOT, "profiles", "batch_allpairs_512.valu.json")
COUNT_VALU = os.path.join(ROOT, "profiles", "count_cooptimal_batch_4096_counts.valu.json")
COUNT_SOURCES = ["paper_2412_21103_amd/csrc/nw_common.h", "paper_2412_21103_amd/csrc/nw_coopt.hip"]


def kernel_hash(sources) -> str:
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def traffic_record(path, sources):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None if the kernel sources changed since the counters were taken."""
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_hash") != kernel_hash(sources):
        return None
    return rec.get("hbm_bytes_per_launch")


def valu_record(path, sources):
    """Measured VALU instructions per cell and VALU busy fraction from a
    committed rocprofv3 counter summary (None if the sources changed)."""
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_hash") != kernel_hash(sources):
        return None
    return {k: rec.get(k) for k in ("valu_lane_instr_per_cell", "valu_busy", "salu_instr_per_cell", "source")}


def _cpu_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def _events_timed(call, warmup, steps, sync, profile=True):
    """W warm-up calls, then K calls each bracketed by HIP events on the
    current stream; returns (wall ms per step, [event ms per step], kernel
    profile of the timed calls)."""
    import torch

    import paper_2412_21103_amd as nwp
    for _ in range(warmup):
        call()
    sync()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    if profile:
        nwp.profile_begin()
    sync()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record()
        call()
        e1.record()
    sync()
    t1 = time.perf_counter()
    prof = nwp.profile_end() if profile else {}
    return (t1 - t0) * 1e3 / steps, [e0.elapsed_time(e1) for e0, e1 in ev], prof


def _stats(ms):
    import statistics
    return {"median_ms": round(statistics.median(ms), 4), "min_ms": round(min(ms), 4),
            "max_ms": round(max(ms), 4)}


def bench_band_batch(args):
    """The learned-band workload (the metric's configuration): 8192 pairs of
    lengths 1,000..20,000, divergence 1..30%, indel fraction 5..50%, scores and
    paths.  Three arms on the same inputs: (i) full DP, (ii) the certified band
    from the best constant starting half-width (chosen on the training pairs
    by wall time) -- the method without the network -- and (iii) the learned
    band, its margin chosen the same way.  The headline is arm (iii); every arm is compared
    with arm (i) on every score and path byte, and arm (iii) with the CPU
    oracle on the cpu_baseline sample.  A reference arm starts every test pair
    at its own path's excursion (from arm (i)'s paths): what an exact width
    predictor would give."""
    import ctypes

    import numpy as np
    import torch

    import paper_2412_21103_amd as nwp
    from paper_2412_21103_amd import band_model
    from workloads import config_band_batch, pack_pairs

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(0)
    npairs = args.band_pairs
    ntrain = max(npairs // 2, 1)
    t = lambda x, dt: torch.from_numpy(np.ascontiguousarray(x, dtype=dt)).to(dev)

    print(f"bench: learned band, generating {npairs} + {ntrain} pairs", file=sys.stderr, flush=True)
    test_pairs = config_band_batch(npairs=npairs)
    train_pairs = config_band_batch(seed=5100, npairs=ntrain)

    class Batch:
        def __init__(self, pairs):
            pool, ao, al, bo, bl = pack_pairs(pairs)
            self.host = (pool, ao, al, bo, bl)
            self.n = len(pairs)
            self.max_len = int(max(al.max(), bl.max()))
            self.d = [t(pool, np.uint8), t(ao, np.int64), t(al, np.int32), t(bo, np.int64), t(bl, np.int32)]
            caps = al.astype(np.int64) + bl.astype(np.int64)
            self.poff_h = np.concatenate([[0], np.cumsum(caps)[:-1]]).astype(np.int64)
            self.poff = t(self.poff_h, np.int64)
            self.cells = float((al.astype(np.float64) * bl.astype(np.float64)).sum())
            self.scores = torch.empty(self.n, dtype=torch.int32, device=dev)
            self.paths = torch.empty(int(caps.sum()), dtype=torch.uint8, device=dev)
            self.plen = torch.empty(self.n, dtype=torch.int32, device=dev)
            self.w_used = torch.empty(self.n, dtype=torch.int32, device=dev)
            self.status = torch.empty(self.n, dtype=torch.uint8, device=dev)
            self.swept = torch.empty(self.n, dtype=torch.int64, device=dev)
            self.swept_so = torch.empty(self.n, dtype=torch.int64, device=dev)

    test, train = Batch(test_pairs), Batch(train_pairs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, _, _, t_path = band_model.features_and_labels(*train.d, train.max_len, label="path")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    mlp, hist = band_model.train(x, t_path, epochs=200, batch=256, lr=3e-3, tau=0.9, seed=1)
    t2 = time.perf_counter()
    # the network the doubling rule needs: trained on the certified width
    _, _, _, t_cert = band_model.features_and_labels(*train.d, train.max_len, label="cert")
    mlp_cert, hist_cert = band_model.train(x, t_cert, epochs=200, batch=256, lr=3e-3, tau=0.9, seed=1)
    print(f"bench: labels {t1 - t0:.2f} s, training {t2 - t1:.2f} s, loss {hist[0]:.3f} -> {hist[-1]:.4f}",
          file=sys.stderr, flush=True)
    del x, t_path, t_cert

    L = nwp.lib()
    sc = nwp.Scoring(*nwp.PAPER_SCORING)
    stream = torch.cuda.current_stream()
    vp = ctypes.c_void_p
    ptr = lambda x: vp(x.data_ptr()) if x is not None else vp(0)
    frac = 0.5
    margin = 0.5       # on the path excursion (widening); replaced by the best on the training pairs
    margin_cert = 0.1  # on the certified width (doubling)
    ws_bytes = max(nwp.learned_workspace_size(test.n, test.max_len), nwp.batch_workspace_size(test.n, test.max_len))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)

    def full(B):
        st = L.nw_align_batch(B.n, *[ptr(v) for v in B.d], B.max_len, sc, 0, ptr(B.scores), ptr(B.paths),
                              ptr(B.poff), ptr(B.plen), ptr(ws), ws_bytes, vp(stream.cuda_stream))
        if st != 0:
            raise nwp.NWError(st, "nw_align_batch")

    def const(B, w0, flags=0):
        st = L.nw_align_batch_banded(B.n, *[ptr(v) for v in B.d], B.max_len, sc, flags, vp(0), int(w0),
                                     ctypes.c_float(frac), ptr(B.scores), ptr(B.paths), ptr(B.poff), ptr(B.plen),
                                     ptr(B.w_used), ptr(B.status), ptr(B.swept), ptr(B.swept_so), ptr(ws), ws_bytes,
                                     vp(stream.cuda_stream))
        if st != 0:
            raise nwp.NWError(st, "nw_align_batch_banded")

    def exact(B, w_init, flags=0):
        # every pair starts at its own optimal path's excursion: the start an
        # exact width predictor would give (a reference for the learned one)
        st = L.nw_align_batch_banded(B.n, *[ptr(v) for v in B.d], B.max_len, sc, flags, ptr(w_init), 0,
                                     ctypes.c_float(frac), ptr(B.scores), ptr(B.paths), ptr(B.poff), ptr(B.plen),
                                     ptr(B.w_used), ptr(B.status), ptr(B.swept), ptr(B.swept_so), ptr(ws), ws_bytes,
                                     vp(stream.cuda_stream))
        if st != 0:
            raise nwp.NWError(st, "nw_align_batch_banded")

    def learned(B, net=None, mg=None, flags=0):
        net = mlp if net is None else net
        mg = margin if mg is None else mg
        st = L.nw_align_batch_learned(B.n, *[ptr(v) for v in B.d], B.max_len, sc, flags, ctypes.byref(net.state),
                                      ctypes.c_float(mg), ctypes.c_float(frac), ptr(B.scores), ptr(B.paths),
                                      ptr(B.poff), ptr(B.plen), ptr(B.w_used), ptr(B.status), ptr(B.swept),
                                      ptr(B.swept_so), ptr(ws), ws_bytes, vp(stream.cuda_stream))
        if st != 0:
            raise nwp.NWError(st, "nw_align_batch_learned")

    sync = torch.cuda.synchronize

    # arm (ii): the best constant starting half-width on the training pairs, by wall time
    print("bench: choosing the constant starting half-width on the training pairs", file=sys.stderr, flush=True)
    DBL = 0x4  # NW_BAND_DOUBLING
    w0_ms, w0_ms_dbl = {}, {}
    for w0 in [0, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096]:
        w0_ms[w0] = min(_events_timed(lambda: const(train, w0), 1, 2, sync, profile=False)[1])
        w0_ms_dbl[w0] = min(_events_timed(lambda: const(train, w0, DBL), 1, 2, sync, profile=False)[1])
    w0_best = min(w0_ms, key=w0_ms.get)
    # the learned arm's margin, chosen the same way: by wall time on the training pairs
    mg_ms = {mg: min(_events_timed(lambda: learned(train, mlp, mg), 1, 2, sync, profile=False)[1])
             for mg in (0.25, 0.5, 1.0, 2.0)}
    margin = min(mg_ms, key=mg_ms.get)
    w0_best_dbl = min(w0_ms_dbl, key=w0_ms_dbl.get)

    def snapshot(B):
        return (B.scores.clone(), B.paths.clone(), B.plen.clone(), B.w_used.clone(), B.status.clone(),
                B.swept.clone(), B.swept_so.clone())

    # identical scores, lengths and every path byte (compared on the device)
    plen_idx = {}

    def same(a, ref):
        s, p, pl = a[0], a[1], a[2]
        s_ref, p_ref, pl_ref = ref[0], ref[1], ref[2]
        if not (torch.equal(s, s_ref) and torch.equal(pl, pl_ref)):
            return False
        if "idx" not in plen_idx:
            pl64 = pl_ref.to(torch.int64)
            starts = torch.repeat_interleave(test.poff, pl64)
            base = torch.repeat_interleave(torch.cumsum(pl64, 0) - pl64, pl64)
            plen_idx["idx"] = starts + torch.arange(int(pl64.sum()), device=dev) - base
        idx = plen_idx["idx"]
        return bool(torch.equal(p[idx], p_ref[idx]))

    W, K = args.warmup, args.steps
    print("bench: arm (i) full DP", file=sys.stderr, flush=True)
    wall_f, ms_f, prof_f = _events_timed(lambda: full(test), W, K, sync)
    ref = snapshot(test)
    w_exact, _ = nwp.path_labels(test.paths, test.poff, test.plen, test.d[2], test.d[4])
    print("bench: reference arm, every pair started at its own path's excursion", file=sys.stderr, flush=True)
    wall_x, ms_x, prof_x = _events_timed(lambda: exact(test, w_exact), W, max(K // 2, 1), sync)
    out_x = snapshot(test)
    print(f"bench: arm (ii) certified band from the constant w0 = {w0_best}", file=sys.stderr, flush=True)
    wall_c, ms_c, prof_c = _events_timed(lambda: const(test, w0_best), W, K, sync)
    out_c = snapshot(test)
    print("bench: doubling arms", file=sys.stderr, flush=True)
    wall_cd, ms_cd, prof_cd = _events_timed(lambda: const(test, w0_best_dbl, DBL), W, max(K // 2, 1), sync)
    out_cd = snapshot(test)
    wall_ld, ms_ld, prof_ld = _events_timed(lambda: learned(test, mlp_cert, margin_cert, DBL), W, max(K // 2, 1), sync)
    out_ld = snapshot(test)
    print("bench: arm (iii) learned band", file=sys.stderr, flush=True)
    wall_l, ms_l, prof_l = _events_timed(lambda: learned(test), W, K, sync)
    out_l = snapshot(test)
    exact_c, exact_l = same(out_c, ref), same(out_l, ref)
    exact_x = same(out_x, ref)
    exact_dbl = same(out_cd, ref) and same(out_ld, ref)

    def arm(name, wall, ms, prof, out, kernel):
        d = {"wall_ms_per_step": round(wall, 3), **_stats(ms),
             "effective_gcups": round(test.cells / (wall * 1e-3) / 1e9, 1)}
        if out is not None:
            st = out[4].cpu().numpy()
            swept = float(out[5].sum())
            d.update({"computed_gcups": round(swept / (wall * 1e-3) / 1e9, 1),
                      "cells_swept_frac": round(swept / test.cells, 4),
                      "certified_first_pass": round(float(np.mean(st & 1)), 4),
                      "extra_passes_mean": round(float(np.mean((st >> 1) & 31)), 3),
                      "full_grid_frac": round(float(np.mean((st & 0x40) != 0)), 4)})
        k = kernel_ms(prof, kernel)
        if k:
            d["kernel"] = kernel
            d["kernel_ms"] = round(k, 4)
            if kernel == "nw_batch_banded" and prof.get(PROBE_KERNEL):
                d["probe_kernel_ms"] = round(kernel_ms(prof, PROBE_KERNEL), 4)
        return d

    res_full = arm("full", wall_f, ms_f, prof_f, None, "nw_batch")
    res_const = arm("const", wall_c, ms_c, prof_c, out_c, "nw_batch_banded")
    res_learned = arm("learned", wall_l, ms_l, prof_l, out_l, "nw_batch_banded")
    res_const["w0"] = w0_best
    res_learned["margin_search_train_ms"] = {str(k): round(v, 2) for k, v in mg_ms.items()}
    res_const["w0_search_train_ms"] = {str(k): round(v, 2) for k, v in w0_ms.items()}
    res_dbl_const = arm("dbl_const", wall_cd, ms_cd, prof_cd, out_cd, "nw_batch_banded")
    res_dbl_const["w0"] = w0_best_dbl
    res_dbl_const["w0_search_train_ms"] = {str(k): round(v, 2) for k, v in w0_ms_dbl.items()}
    res_dbl_learned = arm("dbl_learned", wall_ld, ms_ld, prof_ld, out_ld, "nw_batch_banded")
    res_exact = arm("exact", wall_x, ms_x, prof_x, out_x, "nw_batch_banded")
    res_exact["bit_exact_vs_full_dp"] = exact_x

    # roofline of the banded kernel in the learned arm: computed cells per launch
    # roofline of the banded kernel in the learned arm: the cells of the passes
    # with directions at FILL_OPS_PER_CELL, those of score-only passes at
    # SCORE_OPS_PER_CELL (and again at the 7 and 5 operations per cell the
    # scope counts name)
    kb_ms = kernel_ms(prof_l, "nw_batch_banded")
    swept_cells = float(out_l[5].sum())
    so_cells = float(out_l[6].sum())
    dir_cells = swept_cells - so_cells
    ops = FILL_OPS_PER_CELL * dir_cells + SCORE_OPS_PER_CELL * so_cells
    roof = alu_roofline(BAND_KERNEL_LABEL, ops, kb_ms, 1)
    if roof:
        roof.pop("ops_per_cell")
        roof.update({"cells_with_directions": dir_cells, "cells_score_only": so_cells,
                     "ops_per_cell": {"with_directions": FILL_OPS_PER_CELL, "score_only": SCORE_OPS_PER_CELL}})
        roof["traffic"] = traffic_record(BAND_COUNTERS, BAND_SOURCES)
        ops_scope = 7 * dir_cells + 5 * so_cells
        roof["frac_at_scope_counts"] = round(ops_scope / (kb_ms * 1e-3) / 1e12 / PEAK_INT32_TOPS, 4)
        roof["valu"] = valu_record(BAND_VALU, BAND_SOURCES)

    cpu = exact_oracle = None
    if not args.no_cpu_baseline:
        import oracle
        nt = oracle.max_threads()
        pool, ao, al, bo, bl = test.host
        cum = np.cumsum(al.astype(np.float64) * bl.astype(np.float64))
        target_cells = nt * 7e9  # about 12 s at the oracle's usual rate per thread
        P = int(max(1, min(test.n, np.searchsorted(cum, target_cells) + 1)))
        sub_cells = float(cum[P - 1])
        print(f"bench: CPU oracle on the first {P} pairs ({nt} threads)", file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        s_ref, p_ref = oracle.align_batch(pool, ao[:P], al[:P], bo[:P], bl[:P], oracle.PAPER_SCORING, nthreads=nt)
        c1 = time.perf_counter()
        s_gpu = out_l[0][:P].cpu().numpy()
        pl = out_l[2][:P].cpu().numpy()
        pg = out_l[1].cpu().numpy()
        exact_oracle = bool((s_gpu == s_ref).all() and all(
            np.array_equal(pg[test.poff_h[i]:test.poff_h[i] + pl[i]], p_ref[i]) for i in range(P)))
        cpu = {"value": round(sub_cells / (c1 - c0) / 1e9, 4), "unit": "GCUPS", "cores": nt, "kind": "oracle",
               "sample": f"the first {P} of the {test.n} pairs ({sub_cells:.4g} cells), full DP with scores and "
                         f"paths, OpenMP over pairs, {round(c1 - c0, 2)} s; bit-exact against the learned band: "
                         f"{exact_oracle}", **_cpu_info()}

    config = {"workload": f"band_batch_{npairs}", "pairs": npairs, "full_equivalent_cells": test.cells,
              "scoring": list(nwp.PAPER_SCORING), "traceback": True, "margin": margin, "fallback_frac": frac,
              "growth": "widen a failed band to the width its score certifies",
              "label": "w_path (excursion of the full-DP path beyond the straight band)",
              "learned_band": res_learned, "full_dp": res_full, "constant_band": res_const,
              "speedup_learned_vs_full_dp": round(wall_f / wall_l, 3),
              "speedup_learned_vs_constant_band": round(wall_c / wall_l, 3),
              "exact_width_start": {**res_exact, "label": "w_init = each test pair's own w_path, from the "
                                    "full-DP paths (the start an exact predictor would give; a reference)",
                                    "learned_vs_exact_wall": round(wall_l / wall_x, 3)},
              "doubling": {"label": "w_cert", "margin": margin_cert, "learned_band": res_dbl_learned,
                           "constant_band": res_dbl_const,
                           "speedup_learned_vs_constant_band": round(wall_cd / wall_ld, 3),
                           "bit_exact_vs_full_dp": exact_dbl},
              "bit_exact_learned_vs_full_dp": exact_l, "bit_exact_constant_vs_full_dp": exact_c,
              "bit_exact_vs_oracle_sample": exact_oracle,
              "train_pairs": ntrain, "train_s": round(t2 - t1, 3), "label_dp_s": round(t1 - t0, 3),
              "train_loss": [round(hist[0], 4), round(hist[-1], 4)],
              "train_loss_cert": [round(hist_cert[0], 4), round(hist_cert[-1], 4)]}
    return common_fields(args, test.cells / (wall_l * 1e-3) / 1e9, wall_l, config, roof, cpu)


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


# The banded launch with paths runs its score-only first passes in a launch of
# their own first; the banded kernel's time is the two together.
PROBE_KERNEL = "nw_batch_banded_probe"
BAND_KERNEL_LABEL = "nw_batch_banded (+ nw_batch_banded_probe)"


def kernel_ms(prof, kernel):
    """Mean per-call time of `kernel` (HIP events around each launch); for the
    banded kernel with paths, plus its probe launch's."""
    k = prof.get(kernel)
    if not k:
        return None
    ms = k[1] / k[0]
    if kernel == "nw_batch_banded" and prof.get(PROBE_KERNEL):
        p = prof[PROBE_KERNEL]
        ms += p[1] / p[0]
    return ms


def alu_roofline(kernel, cells, kernel_ms, ops_per_cell):
    """Algorithmic int32 lane-ops (cells x ops_per_cell) per second of the
    kernel's own time, against the chip's int32 VALU peak."""
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
    """4096 pairs, m in [100, 2000], 5-15% mutated, scores + paths, one call per
    step, as the batch layer is meant to run: the sweep-width cost table
    autotuned on a separate sample of the same distribution, and the call's
    launches captured once into a HIP graph (NW_GRAPH) and replayed.  The
    kernel's own time comes from an eager profiled run beside it."""
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
    vp = ctypes.c_void_p
    ptr = lambda x: vp(x.data_ptr())

    print("bench: autotuning the sweep widths on 512 pairs of another seed", file=sys.stderr, flush=True)
    sample = config_batch(seed=3100, npairs=512)
    sp = pack_pairs(sample)
    table = nwp.autotune(t(sp[0], np.uint8), t(sp[1], np.int64), t(sp[2], np.int32), t(sp[3], np.int64),
                         t(sp[4], np.int32), int(max(sp[2].max(), sp[4].max())))

    def step_on(stream, flags):
        st = L.nw_align_batch(npairs, *[ptr(x) for x in d], max_len, sc, flags, ptr(scores), ptr(paths),
                              ptr(d_poff), ptr(plen), ptr(ws), ws_bytes, vp(stream.cuda_stream))
        if st != 0:
            raise nwp.NWError(st, "nw_align_batch")

    side = torch.cuda.Stream()
    sync = torch.cuda.synchronize
    print("bench: eager calls (kernel time)", file=sys.stderr, flush=True)
    with torch.cuda.stream(side):
        wall_e, ms_e, prof = _events_timed(lambda: step_on(side, 0), args.warmup, args.steps, sync)
        print("bench: graph replays (NW_GRAPH)", file=sys.stderr, flush=True)
        wall_g, ms_g, _ = _events_timed(lambda: step_on(side, 0x2), max(args.warmup, 1), args.steps, sync,
                                        profile=False)
    ms = _stats(ms_g)["median_ms"]
    k = prof.get("nw_batch")
    roof = alu_roofline("nw_batch", cells * FILL_OPS_PER_CELL, k[1] / k[0] if k else None, 1)
    if roof:
        roof["ops_per_cell"] = FILL_OPS_PER_CELL
        roof["frac_at_scope_counts"] = round(7 * cells / (k[1] / k[0] * 1e-3) / 1e12 / PEAK_INT32_TOPS, 4)
        roof["traffic"] = traffic_record(BATCH_COUNTERS, BAND_SOURCES)
        roof["valu"] = valu_record(BATCH_VALU, BAND_SOURCES)
    L.nw_release_caches()
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
              "scoring": list(nwp.PAPER_SCORING), "traceback": True, "bit_exact_vs_oracle": exact,
              "graph": _stats(ms_g), "eager": _stats(ms_e), "autotuned_costs": table,
              "graph_gcups": round(cells / (ms * 1e-3) / 1e9, 1),
              "eager_gcups": round(cells / (_stats(ms_e)["median_ms"] * 1e-3) / 1e9, 1)}
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
    if roof:
        roof["valu"] = valu_record(ALLPAIRS_VALU, BAND_SOURCES)
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
    if roof:
        roof["valu"] = valu_record(COUNT_VALU, COUNT_SOURCES)
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


def bench_long_pair(args, length=65536, oracle_check=True):
    """One long pair (ancestor of `length` bases, 10%-mutated descendant):
    whole nw_align calls (fill + traceback), HIP events per call."""
    import ctypes

    import numpy as np
    import torch

    import paper_2412_21103_amd as nwp
    from workloads import config_long_pair

    print(f"bench: generating the {length}-base pair", file=sys.stderr, flush=True)
    pair = config_long_pair(length=length)
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

    print(f"bench: {m} x {n}, warmup {args.warmup}, timing {args.steps} steps", file=sys.stderr, flush=True)
    wall, ms, prof = _events_timed(step, args.warmup, args.steps, torch.cuda.synchronize)
    cells = m * n
    gpu_score = int(score.item())
    k = int(plen.item())
    gpu_path = path[:k].cpu().numpy()
    fill = prof.get("nw_fill_coop")
    fill_ms = fill[1] / fill[0] if fill else None
    tb = [prof[x] for x in ("nw_tb_walk", "nw_tb_spec", "nw_tb_merge", "nw_tb_fix", "nw_tb_emit") if x in prof]
    walk_ms = sum(v[1] / v[0] for v in tb) if tb else None
    roofline = alu_roofline("nw_fill_coop", cells, fill_ms, FILL_OPS_PER_CELL)
    pipeline = None
    if roofline:
        roofline["traffic"] = traffic_record(COOP_COUNTERS, COOP_SOURCES)
        roofline["frac_at_7_ops_per_cell"] = round(7 * cells / (fill_ms * 1e-3) / 1e12 / PEAK_INT32_TOPS, 4)
        valu = valu_record(COOP_VALU, COOP_SOURCES)
        roofline["valu"] = valu
        # The fill is a pipeline of 128-column strips, each starting at least
        # one hop (64 steps of lane skew + one 32-row group) behind the strip
        # to its left: rows + 63 + (strips - 1) * 96 steps of one strip.  At
        # the measured VALU instructions per cell, a step of 2 columns per
        # lane issues in instr/cell * 2 * 4 cycles; the ratio of that bound
        # to the fill time is the fill's fraction of its critical path.
        strips = (n + 127) // 128
        steps = m + 63 + (strips - 1) * 96
        pipeline = {"strips": strips, "critical_path_steps": steps,
                    "measured_ns_per_step": round(fill_ms * 1e6 / steps, 2)}
        if valu and valu.get("valu_lane_instr_per_cell"):
            issue_ns = valu["valu_lane_instr_per_cell"] * 2 * 4 / 2.4
            pipeline.update({"issue_bound_ns_per_step": round(issue_ns, 2),
                             "critical_path_bound_ms": round(steps * issue_ns * 1e-6, 4),
                             "critical_path_frac": round(steps * issue_ns * 1e-6 / fill_ms, 4)})
    cpu = exact = None
    if oracle_check and not args.no_cpu_baseline:
        import oracle
        print("bench: CPU oracle on the same pair (one thread)", file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        s_ref, p_ref = oracle.align(a, b, oracle.PAPER_SCORING, full_limit_bytes=0)
        c1 = time.perf_counter()
        exact = bool(s_ref == gpu_score and np.array_equal(p_ref, gpu_path))
        cpu = {"value": round(cells / (c1 - c0) / 1e9, 4), "unit": "GCUPS", "cores": 1, "kind": "oracle",
               "sample": f"the whole {m} x {n} pair, score + traceback, two score rows + "
                         f"a direction byte per cell, {round(c1 - c0, 2)} s", **_cpu_info()}
    config = {"workload": f"long_pair_{length}", "m": m, "n": n, "mutation_rate": 0.10,
              "scoring": list(nwp.PAPER_SCORING), "traceback": True, **_stats(ms),
              "fill_ms": round(fill_ms, 4) if fill_ms else None,
              "traceback_ms": round(walk_ms, 4) if walk_ms else None,
              "fill_pipeline": pipeline, "bit_exact_vs_oracle": exact}
    return cells / (wall * 1e-3) / 1e9, wall, config, roofline, cpu


def bench_single(args, length=1024):
    """Two independent random sequences of `length` bases: latency of one
    nw_align call (fill + traceback), HIP events per call.  The DP's critical
    path is m + n - 1 dependent anti-diagonals; each needs at least two
    dependent VALU instructions (the max and the tag clear) of 4 cycles at
    2.4 GHz, which bounds the call from below."""
    import ctypes

    import numpy as np
    import torch

    import paper_2412_21103_amd as nwp
    from workloads import config_single

    p = config_single(length=length)
    a, b = p.a[0], p.b[0]
    m, n = len(a), len(b)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(0)
    da, db = torch.from_numpy(a).to(dev), torch.from_numpy(b).to(dev)
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

    steps = max(args.steps, 20)
    wall, ms, prof = _events_timed(step, max(args.warmup, 3), steps, torch.cuda.synchronize)
    import statistics
    med = statistics.median(ms)
    cp_us = (m + n - 1) * 2 * 4 / 2.4e9 * 1e6
    k = int(plen.item())
    exact = None
    if not args.no_cpu_baseline:
        import oracle
        s_ref, p_ref = oracle.align(a, b, oracle.PAPER_SCORING)
        exact = bool(s_ref == int(score.item()) and np.array_equal(p_ref, path[:k].cpu().numpy()))
    kernels = {name: round(v[1] / v[0] * 1e3, 2) for name, v in prof.items() if v[0]}
    return {"workload": f"single_{length}", "m": m, "n": n, "median_us": round(med * 1e3, 2),
            "min_us": round(min(ms) * 1e3, 2), "wall_us_per_call": round(wall * 1e3, 2),
            "gcups": round(m * n / (med * 1e-3) / 1e9, 2),
            "critical_path_steps": m + n - 1, "critical_path_bound_us": round(cp_us, 2),
            "critical_path_frac": round(cp_us / (med * 1e3), 4), "kernel_us": kernels,
            "bit_exact_vs_oracle": exact}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["band_batch", "long_pair", "single", "batch", "allpairs", "center_star",
                                           "cooptimal"], default="band_batch")
    ap.add_argument("--length", type=int, default=65536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="band_batch only: skip the long-pair and single-pair keys")
    ap.add_argument("--no-band", action="store_true", help="alias of --no-extra for the other workloads")
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
    if args.workload == "long_pair":
        value, ms, config, roof, cpu = bench_long_pair(args, args.length)
        print(json.dumps(common_fields(args, value, ms, config, roof, cpu)), flush=True)
        return 0
    if args.workload == "single":
        d = bench_single(args)
        med = d["median_us"] * 1e-3
        print(json.dumps(common_fields(args, d["gcups"], med, d, None, None)), flush=True)
        return 0
    out = bench_band_batch(args)
    if not (args.no_extra or args.no_band):
        value, ms, config, roof, cpu = bench_long_pair(args)
        out["long_pair"] = {"gcups": round(value, 3), "ms_per_step": round(ms, 4), **config, "roofline": roof,
                            "cpu_baseline": cpu}
        out["single_pair"] = bench_single(args)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
