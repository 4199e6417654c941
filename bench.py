"""Benchmark of the batched Smith-Waterman path on one MI355X.

A step is one pass of the whole hot path over the 1M-pair log-normal workload
(median 280, sigma 0.6, lengths 30-5000, identity 10-90%, 3% indels; BLOSUM62,
gap open 11, extend 1): pack the ASCII residues already resident in HBM, sort
the pairs into work cells, align every pair (score and both coordinates) and
write the results.  The persistent form (one persistent launch over a device
work queue, replayed as a HIP graph) is the headline; the plain per-bucket
launch series is timed beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# VALU peaks of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz instructions per
# second; a packed 16-bit instruction does the work of two cells
PEAK_INT32_TOPS = 256 * 64 * 2.4e9 / 1e12
PEAK_PACKED16_TOPS = 2 * PEAK_INT32_TOPS
ALGO_OPS_PER_CELL = 8  # sub, 2x(sub,max) for E and F, add, max3, running max

# name -> (generator, default pairs, length description)
WORKLOADS = {
    "1m-lognormal280": ("config_1m", 1_000_000, "lognormal median 280 sigma 0.6 clipped 30-5000"),
    "heavy-tail": ("config_batching", 20_000, "95% lognormal median 250 sigma 0.6, 5% uniform 5000-35000"),
    "block-50kx50k": ("config_block", 0, "2000 families, lognormal median 280; candidates share >= 2 6-mers"),
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="1m-lognormal280", choices=sorted(WORKLOADS),
                    help="synthetic workload (the default is the headline one)")
    ap.add_argument("--pairs", type=int, default=0, help="pairs (0: the workload's own size)")
    ap.add_argument("--plain-steps", type=int, default=None)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--rows-per-lane", type=int, default=0)
    ap.add_argument("--inter-max", type=int, default=0)
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--group16-max", type=int, default=0)
    ap.add_argument("--group8-max", type=int, default=0)
    ap.add_argument("--autotune", action="store_true",
                    help="run the library's autotuner on the workload before timing")
    ap.add_argument("--autotune-cache", default=None, metavar="JSON",
                    help="the autotuner's cache of per-bucket choices (read and rewritten)")
    ap.add_argument("--no-graph", action="store_true",
                    help="persistent form launched directly instead of replayed as a HIP graph")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (HBM counter calibration) and exit")
    ap.add_argument("--serve", action="store_true",
                    help="serving benchmark instead: open-loop request arrivals, p50/p99 latency")
    ap.add_argument("--serve-families", type=int, default=20000,
                    help="reference families of 50 members (20000: the 1M-reference serving set)")
    ap.add_argument("--serve-batches", type=int, default=200)
    ap.add_argument("--serve-max-batch", type=int, default=10000)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--c3-shards", type=int, default=8,
                    help="devices the 10M-pair heavy-tailed set is split over; one shard is timed")
    ap.add_argument("--parts", default="c2,c3,serve",
                    help="what the default run measures: c2 (the headline), c3 (a heavy-tail shard), "
                         "serve (serving latency); c3 or serve alone only print that object")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(pairs are independent, so the work would shard by pairs)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2303_01845_amd as sw
    from workloads import proteins as P

    assert torch.cuda.is_available(), "bench needs a GPU"
    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        calibrate_copy(torch, dev, args.calibrate_copy)
        return
    if args.serve:
        res = serve_bench(args, (0.3, 0.6, 0.9))
        print(json.dumps(res), flush=True)
        return
    parts = set(args.parts.split(","))
    sw.lib()
    if "c2" not in parts:
        res = {}
        if "c3" in parts:
            res["c3_shard"] = c3_shard_bench(sw, torch, args)
        if "serve" in parts:
            res["serve"] = serve_bench(args, (0.3, 0.6, 0.9))
        print(json.dumps(res), flush=True)
        return
    if args.rows_per_lane or args.inter_max or args.blocks_per_cu or args.group16_max or args.group8_max:
        sw.set_tuning(args.rows_per_lane, args.inter_max, args.blocks_per_cu, args.group16_max, args.group8_max)
    tuning = sw.get_tuning()

    t0 = time.time()
    gen, default_pairs, lengths_desc = WORKLOADS[args.workload]
    n_pairs = args.pairs or default_pairs
    ps = getattr(P, gen)(n_pairs) if n_pairs else getattr(P, gen)()
    cells = ps.cells()
    log("generated %d pairs, %d sequences, %.3f Gcells in %.1fs" % (ps.n_pairs, ps.n_seqs, cells / 1e9,
                                                                   time.time() - t0))
    ascii_d = torch.from_numpy(ps.ascii).to(dev)
    offs_d = torch.from_numpy(ps.offsets).to(dev)
    pairs_d = torch.from_numpy(ps.pairs).to(dev)
    n_res = ascii_d.numel()
    packed_d = torch.empty(sw.packed_bytes(n_res), dtype=torch.uint8, device=dev)
    out_d = torch.empty((ps.n_pairs, 5), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    sptr = stream.cuda_stream

    import ctypes
    L = sw.lib()
    sc = sw.Scoring(0, 11, 1)

    def step(flags):
        rc = L.sw_pack(ctypes.c_void_p(ascii_d.data_ptr()), n_res, ctypes.c_void_p(packed_d.data_ptr()),
                       packed_d.numel(), ctypes.c_void_p(sptr))
        if rc:
            raise sw.SwError(rc, "sw_pack")
        rc = L.sw_batch_align(ctypes.c_void_p(packed_d.data_ptr()), ctypes.c_void_p(offs_d.data_ptr()),
                              ps.n_seqs, ctypes.c_void_p(pairs_d.data_ptr()), ps.n_pairs, ctypes.byref(sc),
                              ctypes.c_void_p(out_d.data_ptr()), ctypes.c_void_p(sptr), flags)
        if rc:
            raise sw.SwError(rc, "sw_batch_align")

    if args.autotune:
        rc = L.sw_pack(ctypes.c_void_p(ascii_d.data_ptr()), n_res, ctypes.c_void_p(packed_d.data_ptr()),
                       packed_d.numel(), ctypes.c_void_p(sptr))
        if rc:
            raise sw.SwError(rc, "sw_pack")
        chosen, ms, trials = sw.autotune(packed_d, offs_d, pairs_d, 11, 1, reps=2, out=out_d, stream=stream,
                                         cache_path=args.autotune_cache)
        log("autotune chose %s (%.2f ms per call, %d bucket trials)" % (chosen, ms, trials))
        tuning = sw.get_tuning()

    def timed(flags, steps, warmup, label):
        for _ in range(warmup):
            step(flags)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
               torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        sw.timing_read(stream)  # forget earlier timed calls
        torch.cuda.synchronize()
        t = time.perf_counter()
        for e0, e1, e2 in ev:
            e0.record(stream)
            L.sw_pack(ctypes.c_void_p(ascii_d.data_ptr()), n_res, ctypes.c_void_p(packed_d.data_ptr()),
                      packed_d.numel(), ctypes.c_void_p(sptr))
            e1.record(stream)
            rc = L.sw_batch_align(ctypes.c_void_p(packed_d.data_ptr()), ctypes.c_void_p(offs_d.data_ptr()),
                                  ps.n_seqs, ctypes.c_void_p(pairs_d.data_ptr()), ps.n_pairs,
                                  ctypes.byref(sc), ctypes.c_void_p(out_d.data_ptr()), ctypes.c_void_p(sptr),
                                  flags | sw.TIMED)
            if rc:
                raise sw.SwError(rc, "sw_batch_align")
            e2.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        fwd_ms, start_ms, calls = sw.timing_read_passes(stream)
        assert calls == steps, (calls, steps)
        kernel_ms = (fwd_ms + start_ms) / steps
        fwd_ms /= steps
        align_ms = [e1.elapsed_time(e2) for _, e1, e2 in ev]
        pack_ms = [e0.elapsed_time(e1) for e0, e1, _ in ev]
        log("%s: %d steps, wall %.3fs, align %.2f ms (min %.2f), kernel %.2f ms, pack %.3f ms" % (
            label, steps, wall, np.mean(align_ms), np.min(align_ms), kernel_ms, np.mean(pack_ms)))
        return wall, float(np.mean(align_ms)), float(np.mean(pack_ms)), kernel_ms, fwd_ms

    # headline: persistent + graph
    log("warmup + timed persistent form")
    pflags = sw.NO_GRAPH if args.no_graph else sw.PERSISTENT
    wall, align_ms, pack_ms, kernel_ms, fwd_ms = timed(pflags, args.steps, args.warmup, "persistent")
    ms_per_step = wall / args.steps * 1e3
    gcups = cells * args.steps / wall / 1e9
    aps = ps.n_pairs * args.steps / wall

    # sampled parity of the last step against the oracle
    import oracle
    got = out_d.cpu().numpy()
    rng = np.random.default_rng(5)
    sample = np.sort(rng.choice(ps.n_pairs, min(2000, ps.n_pairs), replace=False))
    sub = ps.subset(sample)
    exp = oracle.batch_ascii(sub.ascii, sub.offsets, sub.pairs, 11, 1)
    n_ok = int((got[sample] == exp).all(axis=1).sum())
    log("sampled parity %d/%d" % (n_ok, len(sample)))

    plain_steps = args.plain_steps if args.plain_steps is not None else max(1, args.steps // 2)
    plain = None
    if plain_steps > 0:
        pwall, palign_ms, _, pkernel_ms, _ = timed(sw.PLAIN, plain_steps, 1, "plain")
        pgcups = cells * plain_steps / pwall / 1e9
        plain = {"gcups": round(pgcups, 2), "alignments_per_s": round(ps.n_pairs * plain_steps / pwall, 1),
                 "ms_per_step": round(pwall / plain_steps * 1e3, 3), "align_ms": round(palign_ms, 3),
                 "kernel_ms": round(pkernel_ms, 3), "steps": plain_steps}

    # dominant kernel: the persistent alignment kernel, launched twice per
    # step (forward passes, then start passes), each launch timed by HIP
    # events that the library records on the launch stream around it
    achieved = ALGO_OPS_PER_CELL * cells / (kernel_ms * 1e-3) / 1e12
    R = tuning["rows_per_lane"]
    res = {
        "metric": "GCUPS (cell updates/s, full m*n matrix per pair incl. start-coordinate pass), persistent batched form",
        "value": round(gcups, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16x2+i32",
        "data": "synthetic",
        "config": {"workload": args.workload, "pairs": ps.n_pairs, "sequences": ps.n_seqs,
                   "cells": cells, "scoring": "BLOSUM62 gap_open 11 gap_extend 1",
                   "lengths": lengths_desc,
                   "tuning": tuning},
        "alignments_per_s": round(aps, 1),
        "align_ms": round(align_ms, 3),
        "pack_ms": round(pack_ms, 3),
        "kernel_ms": round(kernel_ms, 3),
        "forward_kernel_ms": round(fwd_ms, 3),
        "gcups_fwd": round(cells / (fwd_ms * 1e-3) / 1e9, 2),
        "gcups_fwd_note": "cells / forward launch time alone (the paper's CUPS counts forward scoring only)",
        "plain": plain,
        "persistent_over_plain": round(gcups / plain["gcups"], 3) if plain else None,
        "parity_sample": "%d/%d bit-exact vs CPU oracle" % (n_ok, len(sample)),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_PACKED16_TOPS, 2),
                     "unit": "TOP/s", "frac": round(achieved / PEAK_PACKED16_TOPS, 4),
                     "traffic": stored_traffic(R, ps.n_pairs) if args.workload == "1m-lognormal280" else None,
                     "kernel": "k_persistent<%d>, %d ops per cell x %d cells per step; two launches per "
                               "step (forward, start), mean launch %.3f ms" % (
                                   R, ALGO_OPS_PER_CELL, cells, kernel_ms / 2),
                     "peak_basis": "packed 16-bit VALU (2 cells per instruction), the arithmetic of the "
                                   "score passes; int32 peak %.2f TOP/s gives frac %.4f" % (
                                       PEAK_INT32_TOPS, achieved / PEAK_INT32_TOPS)},
        "paper_context": "paper: 690.6 M alignments/s and 176.3 TCUPS peak on 20,184 V100 GPUs "
                         "(whole application, multi-node; not a 1-GPU target)",
    }
    if args.workload == "block-50kx50k":
        res["identity"] = identity_bench(sw, torch, ps, packed_d, offs_d, pairs_d, out_d, stream, args)
        res["discovery"] = discovery_bench(sw, torch, ps, packed_d, offs_d, stream, args)
        res["pipeline"] = search_bench(sw, torch, ps, packed_d, offs_d, stream, args, res, ms_per_step, cells)
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(ps, args.cpu_seconds)
    if args.workload == "1m-lognormal280":
        # free the headline workload before the larger ones
        del ascii_d, offs_d, pairs_d, packed_d, out_d, ps
        torch.cuda.empty_cache()
        if "c3" in parts:
            res["c3_shard"] = c3_shard_bench(sw, torch, args)
        if "serve" in parts:
            res["serve"] = serve_bench(args, (0.3, 0.6, 0.9))
    print(json.dumps(res), flush=True)


def c3_shard_bench(sw, torch, args):
    """One GPU's share of the 10M-pair heavy-tailed batching set: its chunks
    (65,536 pairs each) assigned longest-first to --c3-shards devices by their
    cost, the first shard generated, packed and aligned in one persistent
    call (one untimed call first), timed by HIP events; results of a sample
    of short and long pairs checked against the oracle.  The projected time
    of the whole set on that many devices is the largest shard's cost at
    this shard's rate."""
    import ctypes
    import oracle
    from workloads import proteins as P
    G = args.c3_shards
    t0 = time.time()
    shards, load, cost = P.c3_lpt_shards(G)
    ps = P.c3_shard(shards[0])
    cells = ps.cells()
    L = ps.lengths().astype(np.int64)
    m, n = L[ps.pairs[:, 0]], L[ps.pairs[:, 1]]
    long_ = np.maximum(m, n) > 4096
    log("c3 shard: %d of %d chunks, %d pairs (%d over 4096 residues), %.4g cells, generated in %.1fs" % (
        len(shards[0]), len(cost), ps.n_pairs, int(long_.sum()), cells, time.time() - t0))
    dev = torch.device("cuda:0")
    ascii_d = torch.from_numpy(ps.ascii).to(dev)
    offs_d = torch.from_numpy(ps.offsets).to(dev)
    pairs_d = torch.from_numpy(ps.pairs).to(dev)
    packed_d = torch.empty(sw.packed_bytes(ascii_d.numel()), dtype=torch.uint8, device=dev)
    out_d = torch.empty((ps.n_pairs, 5), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    sptr = ctypes.c_void_p(stream.cuda_stream)
    Lb = sw.lib()
    sc = sw.Scoring(0, 11, 1)
    rc = Lb.sw_pack(ctypes.c_void_p(ascii_d.data_ptr()), ascii_d.numel(), ctypes.c_void_p(packed_d.data_ptr()),
                    packed_d.numel(), sptr)
    if rc:
        raise sw.SwError(rc, "sw_pack")
    del ascii_d

    def call(flags):
        rc = Lb.sw_batch_align(ctypes.c_void_p(packed_d.data_ptr()), ctypes.c_void_p(offs_d.data_ptr()), ps.n_seqs,
                               ctypes.c_void_p(pairs_d.data_ptr()), ps.n_pairs, ctypes.byref(sc),
                               ctypes.c_void_p(out_d.data_ptr()), sptr, flags)
        if rc:
            raise sw.SwError(rc, "sw_batch_align")

    log("c3 shard: untimed call")
    call(sw.PERSISTENT)
    torch.cuda.synchronize()
    sw.timing_read(stream)
    log("c3 shard: timed call")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t = time.perf_counter()
    e0.record(stream)
    call(sw.PERSISTENT | sw.TIMED)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    call_ms = e0.elapsed_time(e1)
    fwd_ms, start_ms, _ = sw.timing_read_passes(stream)
    got = out_d.cpu().numpy()
    # oracle sample: 400 short pairs, the 2 costliest long pairs and 6 more
    rng = np.random.default_rng(17)
    short_idx = np.flatnonzero(~long_)
    long_idx = np.flatnonzero(long_)
    top = long_idx[np.argsort((m * n)[long_idx])[-2:]]
    rest = np.setdiff1d(long_idx, top)
    pick = np.sort(np.concatenate([rng.choice(short_idx, min(400, len(short_idx)), replace=False), top,
                                   rng.choice(rest, min(6, len(rest)), replace=False)]))
    sub = ps.subset(pick)
    tc = time.perf_counter()
    exp = oracle.batch_ascii(sub.ascii, sub.offsets, sub.pairs, 11, 1, threads=len(os.sched_getaffinity(0)))
    n_ok = int((got[pick] == exp).all(axis=1).sum())
    log("c3 shard: %.1f ms per call (forward %.1f, start %.1f), %.1f GCUPS; oracle sample %d/%d in %.1fs" % (
        call_ms, fwd_ms, start_ms, cells / (call_ms * 1e-3) / 1e9, n_ok, len(pick), time.perf_counter() - tc))
    kernel_ms = fwd_ms + start_ms
    achieved = ALGO_OPS_PER_CELL * cells / (kernel_ms * 1e-3) / 1e12
    wide = float((m * n)[long_].sum()) / cells
    out = {
        "workload": "heavy-tail 10M pairs, LPT shard 1 of %d (chunks of 65,536 pairs assigned longest-first "
                    "by sum of squared query lengths)" % G,
        "chunks": shards[0], "pairs": ps.n_pairs, "long_pairs": int(long_.sum()), "cells": cells,
        "cells_share_over_4096": round(wide, 4),
        "ms": round(call_ms, 2), "wall_ms": round(wall * 1e3, 2),
        "gcups": round(cells / (call_ms * 1e-3) / 1e9, 2),
        "alignments_per_s": round(ps.n_pairs / (call_ms * 1e-3), 1),
        "forward_kernel_ms": round(fwd_ms, 2), "start_kernel_ms": round(start_ms, 2),
        "gcups_fwd": round(cells / (fwd_ms * 1e-3) / 1e9, 2),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_INT32_TOPS, 2),
                     "unit": "TOP/s", "frac": round(achieved / PEAK_INT32_TOPS, 4),
                     "peak_basis": "int32 VALU: %.1f%% of the cells are in pairs over 4,096 residues, whose "
                                   "passes run in packed 16-bit cells up to the first super-strip where a "
                                   "value passes 16 bits and in int32 from there; against the packed 16-bit "
                                   "peak %.2f TOP/s the fraction is %.4f" % (
                                       100 * wide, PEAK_PACKED16_TOPS, achieved / PEAK_PACKED16_TOPS)},
        "projected_full_set_s": round(call_ms * 1e-3 * float(load.max()) / float(load[0]), 2),
        "projected_note": "the whole 10M-pair set on %d GPUs: the largest shard's cost at this shard's rate "
                          "(no transfer or collective time)" % G,
        "parity_sample": "%d/%d bit-exact vs CPU oracle (400 short, the 2 costliest and 6 more long pairs)" % (
            n_ok, len(pick)),
    }
    del packed_d, offs_d, pairs_d, out_d
    torch.cuda.empty_cache()
    return out


def identity_bench(sw, torch, ps, packed_d, offs_d, pairs_d, out_d, stream, args):
    """The identity / coverage pass (sw_identity, thresholds 0.30 and 0.70)
    over the aligned block workload: HIP-event time per call, the cells of the
    boxes it sweeps, the kept count, and a sample against the oracle."""
    import oracle
    rec = torch.empty((ps.n_pairs, 4), dtype=torch.int32, device=out_d.device)
    for _ in range(2):
        sw.identity(packed_d, offs_d, packed_d, offs_d, pairs_d, out_d, 11, 1, 300, 700, flags=sw.VALIDATE,
                    out=rec, stream=stream)
    steps = max(3, args.steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        sw.identity(packed_d, offs_d, packed_d, offs_d, pairs_d, out_d, 11, 1, 300, 700, out=rec, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    sw.check(stream)
    ms = e0.elapsed_time(e1) / steps
    a = out_d.cpu().numpy()
    got = rec.cpu().numpy()
    box = int(((a[:, 2] - a[:, 1] + 1).astype(np.int64) * (a[:, 4] - a[:, 3] + 1))[a[:, 0] > 0].sum())
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(ps.n_pairs, min(1000, ps.n_pairs), replace=False))
    sub = ps.subset(sample)
    exp_aln = oracle.batch_ascii(sub.ascii, sub.offsets, sub.pairs, 11, 1)
    t = time.perf_counter()
    exp = oracle.identity_ascii(sub.ascii, sub.offsets, sub.pairs, exp_aln, 11, 1, 300, 700)
    cpu_s = time.perf_counter() - t
    sa = exp_aln
    sample_cells = int(((sa[:, 2] - sa[:, 1] + 1).astype(np.int64) * (sa[:, 4] - sa[:, 3] + 1))[sa[:, 0] > 0].sum())
    n_ok = int((got[sample] == exp).all(axis=1).sum())
    # the same filter, sweeping only the pairs whose coverage passes
    rec2 = torch.empty_like(rec)
    sw.identity(packed_d, offs_d, packed_d, offs_d, pairs_d, out_d, 11, 1, 300, 700,
                flags=sw.VALIDATE | sw.COVERAGE_FIRST, out=rec2, stream=stream)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        sw.identity(packed_d, offs_d, packed_d, offs_d, pairs_d, out_d, 11, 1, 300, 700, flags=sw.COVERAGE_FIRST,
                    out=rec2, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    sw.check(stream)
    ms_cf = e0.elapsed_time(e1) / steps
    got2 = rec2.cpu().numpy()
    same_keep = bool(np.array_equal(got2[:, 3], got[:, 3]))
    log("identity: %.3f ms per call, %.3f Gcells of boxes, %d of %d kept, sample %d/%d; coverage first %.3f ms "
        "(%d swept, keep flags %s)" % (ms, box / 1e9, int(got[:, 3].sum()), ps.n_pairs, n_ok, len(sample), ms_cf,
                                       int((got2[:, 1] >= 0).sum()), "equal" if same_keep else "DIFFERENT"))
    return {"ms": round(ms, 3), "box_cells": box, "box_gcups": round(box / (ms * 1e-3) / 1e9, 2),
            "kept": int(got[:, 3].sum()), "pairs": ps.n_pairs, "steps": steps,
            "thresholds": "identity >= 0.300, both coverages >= 0.700",
            "parity_sample": "%d/%d equal to the oracle" % (n_ok, len(sample)),
            "coverage_first": {"ms": round(ms_cf, 3), "swept": int((got2[:, 1] >= 0).sum()),
                               "keep_flags_equal": same_keep},
            "oracle_cpu": {"box_gcups": round(sample_cells / cpu_s / 1e9, 4), "cores": 1, "kind": "oracle",
                           "sample": "%d random pairs, %d box cells, %.2f s" % (len(sample), sample_cells, cpu_s)}}


def search_bench(sw, torch, ps, packed_d, offs_d, stream, args, res, align_ms, cells):
    """The whole search on the device (sw_search): discovery of the block
    workload's candidates, their alignment and the identity / coverage filter,
    with the queries in 1, 2 and 4 blocks (with more than one, the next
    block's discovery overlaps the current block, and consecutive blocks run
    on two streams).
    Wall time per call (the call is synchronous), beside the sum of the three
    stages timed alone; the edge count is checked against the stage calls'."""
    nq = (ps.n_seqs + 1) // 2
    qo, ro = offs_d[:nq + 1], offs_d[nq:]
    kept = res["identity"]["kept"]
    cap = kept + 1024
    steps = max(3, args.steps)
    runs = {}
    st = None
    for blocks in (1, 2, 4):
        bq = (nq + blocks - 1) // blocks
        for _ in range(2):
            out = sw.search(packed_d, qo, packed_d, ro, block_queries=bq, edge_cap=cap, stream=stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            out = sw.search(packed_d, qo, packed_d, ro, block_queries=bq, edge_cap=cap, stream=stream)
        wall = (time.perf_counter() - t) / steps
        st = out[3]
        runs[str(blocks)] = {"ms": round(wall * 1e3, 3), "gcups": round(cells / wall / 1e9, 2),
                             "edges_count_equals_stage_calls": st["edges"] == kept}
    stage_ms = res["discovery"]["ms"] + align_ms + res["identity"]["ms"]
    log("search: %s ms per call for 1 / 2 / 4 blocks (%d candidates, %d edges); stages alone %.3f ms" % (
        " / ".join("%.1f" % runs[k]["ms"] for k in ("1", "2", "4")), st["candidates"], st["edges"], stage_ms))
    best = min(runs, key=lambda k: runs[k]["ms"])
    return {"ms": runs[best]["ms"], "blocks": int(best), "by_blocks": runs,
            "candidates": st["candidates"], "edges": st["edges"], "stages_sum_ms": round(stage_ms, 3),
            "stages": "sw_search: sw_discover per query block on one stream, then each block's sw_align_sets, "
                      "sw_identity and edge compaction on one of two more, alternately; stages_sum_ms adds the "
                      "three stages timed alone (the alignment including packing)",
            "steps": steps}


def discovery_bench(sw, torch, ps, packed_d, offs_d, stream, args):
    """Candidate discovery (sw_discover, k = 6, >= 2 shared) of the block
    workload's 50k queries against its 50k references, on the resident packed
    set: wall time per call (the call is synchronous), and the candidate set
    checked against the one the workload generator built."""
    import oracle
    nq = (ps.n_seqs + 1) // 2
    qo, ro = offs_d[:nq + 1], offs_d[nq:]
    cap = ps.n_pairs + 1024
    pairs = torch.empty((cap, 2), dtype=torch.int32, device=offs_d.device)
    shared = torch.empty(cap, dtype=torch.int32, device=offs_d.device)
    L = sw.lib()
    import ctypes
    found = ctypes.c_int64()
    call_args = (ctypes.c_void_p(packed_d.data_ptr()), ctypes.c_void_p(qo.data_ptr()), nq,
                 ctypes.c_void_p(packed_d.data_ptr()), ctypes.c_void_p(ro.data_ptr()), ps.n_seqs - nq, 6, 2,
                 sw.DISCOVER_ALL, ctypes.c_void_p(pairs.data_ptr()), ctypes.c_void_p(shared.data_ptr()), cap,
                 ctypes.byref(found), 0, ctypes.c_void_p(stream.cuda_stream))
    for _ in range(2):
        rc = L.sw_discover(*call_args)
        if rc:
            raise sw.SwError(rc, "sw_discover")
    steps = max(3, args.steps)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        L.sw_discover(*call_args)
    wall = (time.perf_counter() - t) / steps
    n = found.value
    got = pairs[:n].cpu().numpy().astype(np.int64)
    got = got[np.lexsort((got[:, 1], got[:, 0]))]
    gen = ps.pairs.astype(np.int64)
    gen = gen[np.lexsort((gen[:, 1], gen[:, 0]))]
    same = bool(len(got) == len(gen) and np.array_equal(got[:, 0], gen[:, 0]) and
                np.array_equal(got[:, 1] + nq, gen[:, 1]))
    lens = np.diff(ps.offsets)
    windows = int(np.maximum(lens - 5, 0).sum())
    cut = int(ps.offsets[nq])
    t = time.perf_counter()
    oq, _, _ = oracle.discover(ps.ascii[:cut], ps.offsets[:nq + 1], ps.ascii[cut:], ps.offsets[nq:] - cut, 6, 2)
    cpu_s = time.perf_counter() - t
    log("discovery: %.3f ms per call, %d candidates (generator set %s), oracle %.2f s (1 core)" % (
        wall * 1e3, n, "equal" if same else "DIFFERENT", cpu_s))
    return {"ms": round(wall * 1e3, 3), "candidates": n, "kmer_windows": windows,
            "candidates_per_s": round(n / wall, 1), "windows_per_s": round(windows / wall, 1),
            "steps": steps, "k": 6, "min_shared": 2,
            "equals_generator_set": same,
            "oracle_cpu": {"seconds": round(cpu_s, 3), "cores": 1, "kind": "oracle",
                           "candidates": int(len(oq))}}


def serve_bench(args, rhos):
    """Serving: a reference set resident in HBM (families x 50 members), query
    batches of log-uniform size with their k-mer candidates (top 200 per
    query), Poisson arrivals at offered loads 0.3 / 0.6 / 0.9 of the measured
    closed-loop capacity.  Latency = completion - arrival, host buffers in and
    out (PCIe included)."""
    import paper_2303_01845_amd as sw
    from paper_2303_01845_amd.serve import Server, run_open_loop, summarize
    from workloads import proteins as P
    import oracle

    t0 = time.time()
    w = P.serving(n_fam=args.serve_families, per_fam=50, n_batches=args.serve_batches,
                  max_batch=args.serve_max_batch, seed=0)
    Lr = np.diff(w.ref_offsets)
    cells = np.array([int((np.diff(qo)[c[:, 0]].astype(np.int64) * Lr[c[:, 1]]).sum()) for q, qo, c in w.batches])
    log("serve workload: %d refs, %d batches (%d queries, %d candidates, %.3g cells) in %.1fs" % (
        len(Lr), len(w.batches), int(w.sizes.sum()), sum(len(b[2]) for b in w.batches), cells.sum(),
        time.time() - t0))
    refs = sw.Batch(w.ref_ascii, w.ref_offsets)
    srv = Server(refs.packed, refs.offsets, hbm_budget=16 << 30, max_slots=args.serve_slots)
    try:
        n = len(w.batches)
        warm = list(range(min(8, n)))
        run_open_loop(srv, [w.batches[k] for k in warm], np.zeros(len(warm)))
        # capacity: every request offered at time 0, admitted as slots free up
        rec0 = run_open_loop(srv, w.batches, np.zeros(n))
        span0 = max(r["done"] for r in rec0)
        cap = cells.sum() / span0
        log("closed loop: %.1f ms for %d requests, %.1f GCUPS" % (span0 * 1e3, n, cap / 1e9))
        loads = {}
        rng = np.random.default_rng(11)
        for rho in rhos:
            lam = rho * cap / cells.mean()
            arrivals = np.cumsum(rng.exponential(1.0 / lam, n))
            arrivals -= arrivals[0]
            rec = run_open_loop(srv, w.batches, arrivals)
            same = all((r["result"] == r0["result"]).all() for r, r0 in zip(rec, rec0))
            summ = summarize(rec, cells)
            summ["identical_to_closed_loop"] = same
            loads[str(rho)] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()}
            log("load %.1f: p50 %.2f ms p99 %.2f ms, %.1f GCUPS, identical %s" % (
                rho, summ["p50_ms"], summ["p99_ms"], summ["gcups"], same))
            assert same, "results changed between runs"
        # oracle check of a few requests (smallest ones, bounded CPU time)
        order = np.argsort(cells)
        checked = 0
        for k in order[:4]:
            q, qo, cand = w.batches[k]
            asc = np.concatenate([q, w.ref_ascii])
            offs = np.concatenate([qo, w.ref_offsets[1:] + qo[-1]])
            pairs = cand.copy()
            pairs[:, 1] += len(qo) - 1
            exp = oracle.batch_ascii(asc, offs, pairs, 11, 1)
            assert (rec0[k]["result"] == exp).all(), "request %d differs from the oracle" % k
            checked += len(cand)
    finally:
        srv.close()
    last = str(rhos[-1])
    res = {
        "metric": "serve latency p99 at offered load %s (completion - arrival, host buffers)" % last,
        "value": loads[last]["p99_ms"],
        "unit": "ms",
        "n_gpus": 1,
        "higher_is_better": False,
        "data": "synthetic",
        "dtype": "u16x2+i32",
        "config": {"workload": "serve %d references (%d families x 50)" % (len(Lr), args.serve_families),
                   "requests": n,
                   "max_batch": args.serve_max_batch, "slots": args.serve_slots, "hbm_budget_gib": 16,
                   "candidates": "refs sharing >= 2 distinct 6-mers, top 200 per query",
                   "mean_cells_per_request": float(cells.mean())},
        "capacity_gcups": round(cap / 1e9, 2),
        "loads": loads,
        "parity": "every request identical across the closed loop and the open loops; "
                  "%d candidates of the 4 smallest requests bit-exact vs CPU oracle" % checked,
    }
    return res


def calibrate_copy(torch, dev, nbytes):
    """A plain device-to-device copy of a known size, for scaling the HBM
    byte counters (FETCH_SIZE, WRITE_SIZE) of the profiler."""
    src = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log("copied %d bytes 3 times" % (src.numel() * 4))


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_persistent_1m-lognormal280_traffic.md")


def stored_traffic(R, n_pairs):
    """HBM bytes per launch of the persistent kernel as measured by the
    counter runs recorded in the profiles folder, or None when the kernel
    source or the kernel shape changed since they were taken."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    fields = dict(line.split(":", 1) for line in text.splitlines() if line.startswith("- ") and ":" in line)
    fields = {k[2:].strip(): v.strip().strip("`") for k, v in fields.items()}
    src = os.path.join(ROOT, "paper_2303_01845_amd", "csrc", "sw_device.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if (fields.get("kernel source sha256") != digest or fields.get("rows per lane") != str(R)
            or fields.get("pairs") != str(n_pairs)):
        return None
    try:
        return int(fields["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(ps, seconds):
    """The oracle (plain C, as it stands) on a bounded prefix of the same
    workload, all host cores; GCUPS over the same m*n cell count."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    n = 256
    while True:
        sub = ps.subset(np.arange(n))
        t = time.perf_counter()
        oracle.batch_ascii(sub.ascii, sub.offsets, sub.pairs, 11, 1, threads=threads)
        dt = time.perf_counter() - t
        if dt > seconds / 4 or n >= ps.n_pairs:
            break
        n = min(ps.n_pairs, int(n * max(2.0, seconds / max(dt, 1e-3) * 0.9)))
    log("cpu oracle: %d pairs in %.2fs on %d threads" % (n, dt, threads))
    return {"value": round(sub.cells() / dt / 1e9, 4), "unit": "GCUPS", "cores": threads, "kind": "oracle",
            "sample": "first %d of the %d pairs (%.3f Gcells), forward + start pass" % (n, ps.n_pairs,
                                                                                       sub.cells() / 1e9),
            "alignments_per_s": round(n / dt, 1)}


if __name__ == "__main__":
    main()
