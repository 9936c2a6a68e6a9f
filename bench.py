"""Benchmark: GCUPS with traceback of batched read-vs-window affine-gap
alignment on one MI355X (seeded synthetic data).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload config5|config2|config3|config4|multi|mate]

Default workload: the low-similarity batch, 500,000 reads x 150 bp at
60-75% identity against 1,000 bp windows.  `value` is the plain int32
form's GCUPS; the batched form (length classes, packed int16 with int32
re-run, persistent kernels, graph replay, autotuned shapes) runs on the same
data and is reported beside it with its own roofline.  A step is one
soap_dp_align_batch call over the whole batch (fill, traceback and CIGAR of
every task), inputs resident in device memory.  The default run adds the
uneven batch (2,000,000 reads of 36-250 bp) in both forms and a served leg
at the frozen arrival rate with its p50/p99 latency.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GCUPS w/ traceback, batched vs plain kernel; p50/p99 latency at fixed QPS"
SCORING = (1, -3, -5, -2)
OPS_PER_CELL = 14            # 10 score operations + 4 decision comparisons per cell
OPS_PER_CELL_SCORE = 10      # score-only pass: no decision comparisons
# Calls with traceback run two passes: the score recurrences over every
# window cell, then recurrences and decisions over the band cells only, so
# their algorithmic count is 10 per window cell plus 14 per band cell.
PEAK_INT32_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # CUs x SIMDs x lanes x clock = 39.3 T lane-ops/s
PEAK_INT16_TOPS = 2 * PEAK_INT32_TOPS            # packed 2 x int16 per lane

# HBM traffic of one call (the score-pass and decision-pass DP kernels; the
# band and fix-up kernels move a few MB), from two rocprofv3 --pmc runs
# (FETCH_SIZE, WRITE_SIZE; KiB per dispatch, summed over the call's
# kernels) scaled by what the same counters read for a plain 1 GiB device
# copy (FETCH x 2.000, WRITE x 1.000).  Keyed by (workload, form); valid
# only for the kernel sources fingerprinted (any change to them makes
# `traffic` null until the counters are re-taken).
KERNEL_SOURCES = ("api.cpp", "band.h", "band.hip", "batch.h", "batch.hip", "dp_device.h",
                  "dp_i16.hip", "dp_i32.hip", "dp_internal.h")
TRAFFIC = {
    # per call: the score-pass and decision-pass kernels together; the
    # batched entry holds for the class shapes named (the autotuner runs at
    # the start of every bench run and may pick others)
    ("config5", "plain"): {"fingerprint": "701539a1eb9fc68b",
                           "kernel": "dp_i32_kernel<4,38,byte> score pass + decision pass",
                           "fetch_kib": 2051595, "write_kib": 9390437,
                           "fetch_scale": 2.000, "write_scale": 1.000},
    ("config5", "batched"): {"fingerprint": "701539a1eb9fc68b",
                             "kernel": "dp_i16_kernel class 152: 4x38 score pass + 8x19 decision pass",
                             "shapes": {"i16/152": "8x19"},
                             "fetch_kib": 2614460, "write_kib": 11432776,
                             "fetch_scale": 2.000, "write_scale": 1.000},
}


def kernel_fingerprint() -> str:
    import hashlib
    csrc = os.path.join(ROOT, "paper_1302_5507_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(f.encode())
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _entry_holds(t, shapes) -> bool:
    """The counters were taken on these sources and, for the batched form,
    with these class shapes."""
    if t is None or t["fingerprint"] != kernel_fingerprint():
        return False
    want = t.get("shapes")
    return not want or all((shapes or {}).get(k) == v for k, v in want.items())


def traffic_bytes(workload: str, form: str, shapes=None):
    t = TRAFFIC.get((workload, form))
    if not _entry_holds(t, shapes):
        return None
    return int(round((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024))


# VALU wave-instructions of one call's DP kernels (rocprofv3 --pmc
# SQ_INSTS_VALU), same keying and fingerprint rule as TRAFFIC.  The issue
# fraction divides them by what the chip can issue in the measured device
# time of the call: one wave64 VALU instruction per SIMD every 4 cycles.
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4
VALU_INSTS = {
    ("config5", "plain"): {"fingerprint": "701539a1eb9fc68b", "sq_insts_valu": 11069547880},
    ("config5", "batched"): {"fingerprint": "701539a1eb9fc68b", "shapes": {"i16/152": "8x19"},
                             "sq_insts_valu": 8018535566},
}


def valu_issue_frac(workload: str, form: str, kernel_ms: float, shapes=None):
    t = VALU_INSTS.get((workload, form))
    if not _entry_holds(t, shapes):
        return None
    return round(t["sq_insts_valu"] / (kernel_ms * 1e-3 * VALU_ISSUE_PER_S), 4)


WORKLOADS = {
    "config2": ("mate-rescue: 1,000,000 reads x 100 bp vs 250 bp windows from a 1 Mbp random "
                "genome (2% subs, 0.5% indels, 10% random reads)", "config2", "plain"),
    "config3": ("uneven: 2,000,000 reads, n uniform over {36,50,75,100,150,250}, m = n + 160 "
                "(4% subs, 0.5% indels up to 30 bp)", "config3", "batched"),
    "config5": ("low-similarity: 500,000 reads x 150 bp at 60-75% identity vs 1,000 bp windows "
                "from a 1 Mbp random genome (substitutions 0.75 d, indel events 0.05 d of "
                "geometric length <= 50, d = 1 - identity)", "config5", "plain"),
}


def cpu_baseline(w, tasks: int, scoring=SCORING):
    import oracle
    idx = np.arange(min(tasks, w.n_tasks))
    cells = int(np.dot(w.read_len[idx].astype(np.int64), w.ref_len[idx].astype(np.int64)))
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    oracle.align_workload(w, oracle.scoring(*scoring), idx=idx, n_threads=threads)
    dt = time.perf_counter() - t0
    what = "all" if idx.size == w.n_tasks else f"first {idx.size:,}"
    # one core on a fixed 20,000-task prefix
    idx1 = np.arange(min(20_000, w.n_tasks))
    cells1 = int(np.dot(w.read_len[idx1].astype(np.int64), w.ref_len[idx1].astype(np.int64)))
    t1 = time.perf_counter()
    oracle.align_workload(w, oracle.scoring(*scoring), idx=idx1, n_threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": round(cells / dt / 1e9, 4), "unit": "GCUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{what} tasks of the same workload ({cells:.3g} cells), three-table int32 "
                      f"C oracle with traceback, {threads} threads, {dt:.1f} s",
            "single_core": {"value": round(cells1 / dt1 / 1e9, 4), "unit": "GCUPS",
                            "sample": f"first {idx1.size:,} tasks, 1 thread, {dt1:.1f} s"}}


# Frozen arrival rate of the served workload: 0.7 x the capacity measured
# with everything arriving at once (--qps 0: 102,607 requests/s, 2,078
# GCUPS, 3 slots x 131,072 reads), rounded to 2 significant figures.
SERVE_QPS = 72000.0


def serve_bench(args):
    print(json.dumps(serve_run(args, args.qps if args.qps is not None else SERVE_QPS)), flush=True)


def serve_run(args, qps):
    """Served workload: Poisson arrivals of requests of 1..4096 reads
    (log-uniform), reads 50-250 bp over a device-resident 100 Mbp genome.
    With qps 0 the requests all arrive at once, which measures capacity.
    Returns the JSON line as a dict."""
    import torch
    from paper_1302_5507_amd import binding, serving, workloads
    import oracle

    g = workloads.serving_genome()
    gw = torch.from_numpy(binding.pack_words(g).view(np.int32)).cuda()
    pool = workloads.serving_pool(g, args.pool_reads)
    n_total = args.serve_warmup + args.serve_requests
    sizes = workloads.request_sizes(n_total, seed=104)
    reqs = serving.requests_from_pool(pool, sizes)
    srv = serving.Server(gw, n_slots=args.slots, max_tasks=args.slot_tasks, max_n=250, max_m=410,
                         autotune=True, device_bytes=args.device_bytes,
                         align_flags=0 if args.serve_two_pass else binding.FULL_WINDOW)
    # the whole schedule is submitted ahead; the server admits each request
    # at its arrival time (all at once when measuring capacity)
    arr, done, lag = serving.run_open_loop(srv, reqs, qps, seed=104)
    bad = [r.rc for r in reqs if r.rc != 0]
    if bad:
        vals, counts = np.unique(bad, return_counts=True)
        raise RuntimeError(f"{len(bad)} served requests failed: codes {dict(zip(vals.tolist(), counts.tolist()))}; "
                           f"server {srv.stats()}")
    meas = slice(args.serve_warmup, n_total)
    if qps > 0:   # sustained rate over the measured requests
        cells = sum(r.cells for r in reqs[meas])
        span = (done[meas].max() - arr[meas].min()) * 1e-9
    else:         # capacity: everything arrives at once
        cells = sum(r.cells for r in reqs)
        span = (done.max() - arr.min()) * 1e-9
    lat = (done[meas] - arr[meas]) * 1e-6
    # where the time went: queue (arrival to taken into a batch), launch
    # (merge and enqueue), device (until the batch's results are in host
    # memory), retire (hand-off into the request's buffers)
    phases = np.array([r.phases_ns() for r in reqs[meas]], np.float64) * 1e-6
    slow = lat >= np.percentile(lat, 99)
    names = ("queue", "launch", "device", "retire")
    breakdown = {
        "p50": {k: round(float(np.percentile(phases[:, i], 50)), 3) for i, k in enumerate(names)},
        "p99": {k: round(float(np.percentile(phases[:, i], 99)), 3) for i, k in enumerate(names)},
        "slowest_1pct_mean": {k: round(float(phases[slow, i].mean()), 3)
                              for i, k in enumerate(names)},
    }
    # the batches whose enqueue took longest, warm-up included: when (ms
    # after the first measured arrival; negative in the warm-up), how long,
    # and how many requests and reads waited
    taken = np.array([r.stamps.taken_ns for r in reqs], np.int64)
    ntask = np.array([r.n_tasks for r in reqs], np.int64)
    launch_all = np.array([r.stamps.launched_ns - r.stamps.taken_ns for r in reqs], np.float64) * 1e-6
    keys, first, inv = np.unique(taken, return_index=True, return_inverse=True)
    b_launch = launch_all[first]
    b_reqs = np.bincount(inv)
    b_tasks = np.bincount(inv, weights=ntask)
    t_origin = arr[meas].min()
    slow_launches = [{"at_ms": round(float((keys[b] - t_origin) * 1e-6), 1),
                      "launch_ms": round(float(b_launch[b]), 3), "requests": int(b_reqs[b]),
                      "reads": int(b_tasks[b])}
                     for b in np.argsort(-b_launch)[:5]]
    rng = np.random.default_rng(4)
    checked = 0
    for k in rng.choice(np.arange(args.serve_warmup, n_total), size=min(20, args.serve_requests),
                        replace=False):
        r = reqs[k]
        ref = oracle.align_workload(pool, oracle.scoring(*SCORING), idx=r.pool_idx, cigar_stride=500)
        assert np.array_equal(r.score, ref.score) and np.array_equal(r.cigar_len, ref.cigar_len)
        assert np.array_equal(r.ref_begin, ref.ref_begin) and np.array_equal(r.ref_end, ref.ref_end)
        for t, row in enumerate(r.cigar_rows()):
            assert np.array_equal(row, ref.cigar_of(t))
        checked += 1
    st = srv.stats()
    srv.close()
    mean_cells = float(np.mean([r.cells for r in reqs[meas]]))
    line = {
        "metric": METRIC,
        "value": round(cells / span / 1e9, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.serve_requests,
        "warmup": args.serve_warmup,
        "ms_per_step": round(float(np.mean(lat)), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int16+int32",
        "data": "synthetic",
        "config": {"workload": "served: Poisson arrivals of 1-4096-read requests (log-uniform), "
                               "reads 50-250 bp vs n+160 windows in a resident 100 Mbp genome",
                   "qps": qps if qps > 0 else "saturation", "slots": args.slots,
                   "passes": 2 if args.serve_two_pass else 1,
                   "slot_tasks": args.slot_tasks,
                   "requests": args.serve_requests, "mean_cells_per_request": round(mean_cells)},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3),
                       "max": round(float(lat.max()), 3)},
        "latency_phases_ms": breakdown,
        "slowest_launches": slow_launches,
        "achieved_qps": round((args.serve_requests if qps > 0 else n_total) / span, 1),
        "late_submissions": int((lag[meas] > 0).sum()),
        "server": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()},
        "oracle_checked_requests": checked,
    }
    return line


MULTI_DESC = ("multi-candidate: 200,000 reads of 100 or 150 bp, 1 + Poisson(11) candidate "
              "windows each (at most 40; n + 60 bp, random strand, support uniform 1..20) "
              "from a 1 Mbp random genome, the best `ceiling` by support aligned, best and "
              "second best with the best's CIGAR")


def multi_cells(mw, ceiling):
    """Cells of the aligned (read, candidate) pairs and of the final pass
    (every candidate of the generated lists is valid)."""
    k = np.minimum(np.diff(mw.cand_start), ceiling)
    n = mw.read_len.astype(np.int64)
    m = n + 2 * int(mw.params["flank"])
    return int(np.sum(k * n * m)), int(np.sum(np.where(k > 0, n * m, 0)))


def multi_bench(args):
    import torch
    from paper_1302_5507_amd import binding, workloads
    mw = workloads.multi_candidate()
    C = args.ceiling
    al = binding.Aligner(0)
    al.autotune(args.tune_cache)
    dm = binding.DeviceMultiWorkload(mw)
    res = binding.DeviceMultiResult(mw.n_reads, 2 * dm.max_n)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        al.align_multi(dm, C, SCORING, res=res)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        al.align_multi(dm, C, SCORING, res=res)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    s = (time.perf_counter() - t0) / args.steps
    dev_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    out = res.to_host()
    assert np.isin(out["status"], (0, 2)).all(), "unaligned reads in bench"
    cand_cells, final_cells = multi_cells(mw, C)
    ops = OPS_PER_CELL_SCORE * cand_cells + OPS_PER_CELL * final_cells
    achieved = ops / (dev_ms * 1e-3) / 1e12
    line = {
        "metric": "GCUPS over aligned candidate windows (multi-candidate call, effort limit)",
        "value": round(cand_cells / s / 1e9, 2),
        "unit": "GCUPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(s * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int16+int32", "data": "synthetic",
        "config": {"workload": MULTI_DESC, "ceiling": C, "n_reads": mw.n_reads,
                   "n_cands": mw.n_cands, "candidate_cells": cand_cells,
                   "final_cells": final_cells, "scoring": list(SCORING)},
        "reads_per_s": round(mw.n_reads / s, 1),
        "true_window_found": round(float(np.mean(out["best_cand"] == mw.true_cand)), 5),
        "roofline": {
            "bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_INT16_TOPS, 1),
            "unit": "TOP/s", "frac": round(achieved / PEAK_INT16_TOPS, 4), "traffic": None,
            "ops": f"{OPS_PER_CELL_SCORE}/cell score pass + {OPS_PER_CELL}/cell final pass",
            "kernel_ms": round(dev_ms, 3),
        },
    }
    if not args.no_cpu_baseline:
        import oracle
        from oracle import multi as omulti
        R = min(args.cpu_reads, mw.n_reads)
        e = int(mw.cand_start[R])
        threads = oracle.default_threads()
        t0 = time.perf_counter()
        omulti.align_multi(mw.read_codes, mw.read_off[:R], mw.read_len[:R], mw.genome,
                           mw.cand_start[:R + 1], mw.cand_off[:e], mw.cand_len[:e],
                           mw.cand_support[:e], mw.cand_strand[:e], oracle.scoring(*SCORING),
                           dm.max_n, dm.max_m, C, n_threads=threads)
        dt = time.perf_counter() - t0
        k = np.minimum(np.diff(mw.cand_start[:R + 1]), C)
        n = mw.read_len[:R].astype(np.int64)
        cells = int(np.sum(k * n * (n + 2 * int(mw.params["flank"]))))
        line["cpu_baseline"] = {
            "value": round(cells / dt / 1e9, 4), "unit": "GCUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"first {R:,} reads of the same workload ({cells:.3g} candidate cells), "
                      f"multi-candidate oracle, {threads} threads, {dt:.1f} s"}
    print(json.dumps(line), flush=True)
    al.close()


MATE_DESC = ("mate rescue: 1,000,000 pairs of 100 bp ends from a 1 Mbp random genome, "
             "fragments N(500, 50^2), FR orientation, regions for fragments of 425..575 bp "
             "generated on the device (250 bp), unaligned end with 2% subs, 0.5% indels, 10% "
             "random")


def mate_bench(args):
    import torch
    from paper_1302_5507_amd import binding, workloads
    mw = workloads.mate_pairs()
    al = binding.Aligner(0)
    al.autotune(args.tune_cache)
    dm = binding.DeviceMateWorkload(mw)
    res = binding.DeviceMateResult(mw.n_reads, 2 * dm.max_n)
    stream = torch.cuda.current_stream()
    forms = {}
    for name, flags in (("batched", binding.BATCHED), ("plain", binding.PLAIN)):
        for _ in range(args.warmup):
            al.mate_rescue(dm, SCORING, flags=flags, res=res)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        t0 = time.perf_counter()
        for k in range(args.steps):
            ev[k][0].record(stream)
            al.mate_rescue(dm, SCORING, flags=flags, res=res)
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        s = (time.perf_counter() - t0) / args.steps
        out = res.to_host()
        assert np.isin(out["status"], (0, 2)).all(), "unaligned pairs in bench"
        cells = int(np.dot(mw.read_len.astype(np.int64), out["window_len"].astype(np.int64)))
        forms[name] = (s, float(np.mean([a.elapsed_time(b) for a, b in ev])), cells, out)
    s, dev_ms, cells, out = forms["batched"]
    achieved = OPS_PER_CELL * cells / (dev_ms * 1e-3) / 1e12
    line = {
        "metric": "GCUPS w/ traceback, mate rescue with device-side regions",
        "value": round(cells / s / 1e9, 2), "unit": "GCUPS",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(s * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int16+int32", "data": "synthetic",
        "config": {"workload": MATE_DESC, "form": "batched", "n_pairs": mw.n_reads, "cells": cells,
                   "min_frag": mw.v, "max_frag": mw.u, "scoring": list(SCORING)},
        "mate_found": round(float(np.mean(out["window_off"].astype(np.int64) + out["ref_begin"]
                                          == mw.true_pos)), 5),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": round(PEAK_INT16_TOPS, 1), "unit": "TOP/s",
                     "frac": round(achieved / PEAK_INT16_TOPS, 4), "traffic": None,
                     "ops_per_cell": OPS_PER_CELL, "kernel_ms": round(dev_ms, 3)},
        "forms": {f: {"gcups": round(c / fs / 1e9, 2), "ms_per_step": round(fs * 1e3, 3),
                      "device_ms": round(fk, 3)} for f, (fs, fk, c, _) in forms.items()},
    }
    if not args.no_cpu_baseline:
        import oracle
        from oracle import mate as omate
        R = min(args.cpu_pairs, mw.n_reads)
        threads = oracle.default_threads()
        t0 = time.perf_counter()
        ref = omate.rescue(mw.read_codes, mw.read_off[:R], mw.read_len[:R], mw.genome,
                           mw.mate_pos[:R], mw.mate_len[:R], mw.mate_strand[:R], mw.v, mw.u,
                           mw.orientation, oracle.scoring(*SCORING), dm.max_n, n_threads=threads)
        dt = time.perf_counter() - t0
        c = int(np.dot(mw.read_len[:R].astype(np.int64), ref.window_len.astype(np.int64)))
        line["cpu_baseline"] = {
            "value": round(c / dt / 1e9, 4), "unit": "GCUPS", "cores": threads, "kind": "oracle",
            "sample": f"first {R:,} pairs of the same workload ({c:.3g} cells), mate-rescue "
                      f"oracle (regions in Python, C three-table DP), {threads} threads, {dt:.1f} s"}
    print(json.dumps(line), flush=True)
    al.close()


LAYOUT_DESC = ("short reads: 2,000,000 reads of 16 bp and of 32 bp vs n + 160 windows (the "
               "uneven batch's error model), reads stored one after another or word by word "
               "in groups of 32")


def layout_bench(args):
    """The paper's word-interleaved read layout against reads stored one
    after another, on the shapes with 32-64 tasks per wavefront (16 and 32
    bp reads), both forms: device ms per call."""
    import torch
    from paper_1302_5507_amd import binding, workloads
    al = binding.Aligner(0)
    al.autotune(args.tune_cache)
    out = {}
    for n in (16, 32):
        w = workloads.short_reads(n)
        res = binding.DeviceResult(w.n_tasks, 2 * n)
        for inter in (False, True):
            dw = binding.DeviceWorkload(w, interleaved=inter)
            for form, flags in (("plain", binding.PLAIN), ("batched", binding.BATCHED)):
                s, k, host = time_form(al, dw, res, flags, args.steps, args.warmup, SCORING)
                key = f"{n}bp/{form}/{'interleaved' if inter else 'natural'}"
                out[key] = {"gcups": round(w.cells / s / 1e9, 2), "device_ms": round(k, 3)}
                print(f"bench: {key} {out[key]}", file=sys.stderr, flush=True)
            del dw
    shapes = {f"i{p}/{c}": f"{l}x{k}" for p, c, l, k in al.classes() if c <= 32}
    line = {"metric": "device ms per call by read layout", "value": None, "unit": "ms",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "data": "synthetic",
            "config": {"workload": LAYOUT_DESC, "scoring": list(SCORING)},
            "layouts": out, "shapes": shapes}
    print(json.dumps(line), flush=True)
    al.close()


def time_form(al, dw, res, flags, steps, warmup, scoring):
    """Warm up, then time `steps` calls back to back on the current stream:
    (host seconds per call, mean device ms per call from HIP events on the
    stream the library's work is enqueued on, host copy of the outputs)."""
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        al.align(dw, scoring, flags=flags, res=res)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        al.align(dw, scoring, flags=flags, res=res)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    out = res.to_host()
    assert (out["status"] != 1).all() and (out["status"] != 3).all(), "invalid tasks in bench"
    return elapsed / steps, float(np.mean([a.elapsed_time(b) for a, b in ev])), out


def band_cells(w, out, scoring):
    """Cells of the decision pass: each aligned task's read length times the
    window rows [i0, end) that can hold an optimal alignment of score S,
    i0 = max(0, end - n - Dmax), Dmax = 1 + (n S_MA + S_GO - S) // |S_GE|
    (0 when negative); the whole window when S_GE = 0."""
    ma, mi, go, ge = scoring
    n = w.read_len.astype(np.int64)
    ok = np.isin(out["status"], (0, 2))
    S = out["score"].astype(np.int64)
    e = out["ref_end"].astype(np.int64)
    if ge == 0:
        i0 = np.zeros_like(e)
    else:
        x = n * ma + go - S
        dmax = np.where(x < 0, 0, 1 + np.maximum(x, 0) // (-ge))
        i0 = np.maximum(0, e - n - dmax)
    return int(np.sum(np.where(ok, n * (e - i0), 0)))


def align_legs(args, al, w, forms, scoring, score_only=False, full_window=False):
    """Time the requested forms on one workload.  Returns {form: summary}."""
    from paper_1302_5507_amd import binding
    dw = binding.DeviceWorkload(w)
    extra = (binding.SCORE_ONLY if score_only else 0) | (binding.FULL_WINDOW if full_window else 0)
    res = binding.DeviceResult(w.n_tasks, 0 if score_only else 2 * dw.max_n)
    cells_t = w.read_len.astype(np.int64) * w.ref_len.astype(np.int64)
    out = {}
    for form in forms:
        flags = (binding.BATCHED if form == "batched" else binding.PLAIN) | extra
        s, k, host = time_form(al, dw, res, flags, args.steps, args.warmup, scoring)
        redone = host["status"] == binding.TASK_OK_REDONE_INT32
        if form == "plain":
            peak, f32 = PEAK_INT32_TOPS, 1.0
        else:
            # int16 classes at the packed peak, re-run tasks at the int32 one,
            # weighted by their share of the cells
            f32 = float(cells_t[redone].sum() / max(cells_t.sum(), 1))
            peak = 1.0 / ((1.0 - f32) / PEAK_INT16_TOPS + f32 / PEAK_INT32_TOPS)
        if score_only:
            ops, bc = OPS_PER_CELL_SCORE * w.cells, 0
        elif full_window:
            ops, bc = OPS_PER_CELL * w.cells, w.cells
        else:
            bc = band_cells(w, host, scoring)
            ops = OPS_PER_CELL_SCORE * w.cells + OPS_PER_CELL * bc
        achieved = ops / (k * 1e-3) / 1e12
        d = {"gcups": round(w.cells / s / 1e9, 2), "ms_per_step": round(s * 1e3, 3),
             "device_ms": round(k, 3), "achieved_tops": round(achieved, 3),
             "ops_per_step": ops, "band_cells": bc,
             "peak_tops": round(peak, 2), "valu_frac": round(achieved / peak, 4),
             "redone_int32": round(float(redone.mean()), 4),
             "int32_cell_share": round(f32, 4)}
        if form == "batched":
            lengths = sorted(set(int(x) for x in np.unique(w.read_len)))
            shapes = {}
            for prec, cap, lanes, cls_cells in al.classes():
                hit = [n for n in lengths if n <= cap and not any(
                    n <= c for p2, c, _, _ in al.classes() if p2 == prec and c < cap)]
                if hit:
                    shapes[f"i{prec}/{cap}"] = f"{lanes}x{cls_cells}"
            d["shapes"] = shapes
        out[form] = (s, k, d)
    del dw, res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["config4", "multi", "mate", "layout"],
                    default="config5")
    ap.add_argument("--no-extra", action="store_true",
                    help="default workload only: skip the uneven batch and the served leg")
    ap.add_argument("--ceiling", type=int, default=30, help="multi workload: candidates aligned per read")
    ap.add_argument("--cpu-reads", type=int, default=160_000, help="multi workload: oracle sample")
    ap.add_argument("--cpu-pairs", type=int, default=1_000_000, help="mate workload: oracle sample")
    ap.add_argument("--qps", type=float, default=None, help="served workload: arrival rate (0: saturate)")
    ap.add_argument("--slots", type=int, default=3)
    ap.add_argument("--slot-tasks", type=int, default=131072, help="served workload: reads per slot")
    ap.add_argument("--pool-reads", type=int, default=400_000)
    ap.add_argument("--device-bytes", type=int, default=0,
                    help="served workload: device memory the batches in flight share (0: one "
                         "full batch per slot)")
    ap.add_argument("--serve-two-pass", action="store_true",
                    help="served workload: score pass + band pass per batch instead of one pass "
                         "(SOAP_DP_FULL_WINDOW, the default: served batches are short-window "
                         "and launch-bound, where one pass is faster)")
    # about 55 ms of arrivals at 72,000/s: each slot's first few batches
    # enqueue slowly (up to 10 ms), which is start-up, not steady serving
    ap.add_argument("--serve-warmup", type=int, default=4000)
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--form", choices=["plain", "batched", "both"], default="both")
    ap.add_argument("--cpu-tasks", type=int, default=250_000,
                    help="oracle sample: the first tasks of the workload (all threads)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--score-only", action="store_true",
                    help="score and end only (SOAP_DP_SCORE_ONLY), no traceback")
    ap.add_argument("--full-window", action="store_true",
                    help="one pass with decision bits over the whole window "
                         "(SOAP_DP_FULL_WINDOW) instead of score pass + band pass")
    ap.add_argument("--score-scale", type=int, default=1,
                    help="multiply every score by K (the overflow runs: x100 on config3, "
                         "x128 on config5)")
    ap.add_argument("--tune-cache", default=os.environ.get("SOAPDP_TUNE_CACHE"))
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run device-to-device copies of BYTES (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only; the tasks are independent and would be "
              "split across GPUs by task range with no communication, but no multi-GPU run is "
              "made here", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1302_5507_amd import binding, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        # a plain copy of known size: reads and writes BYTES each per launch
        a = torch.empty(args.calibrate_copy // 4, dtype=torch.int32, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": args.calibrate_copy}), flush=True)
        return

    if args.workload == "config4":
        serve_bench(args)
        return
    if args.workload == "multi":
        multi_bench(args)
        return
    if args.workload == "mate":
        mate_bench(args)
        return
    if args.workload == "layout":
        layout_bench(args)
        return
    scoring = tuple(args.score_scale * x for x in SCORING)
    desc, gen, headline = WORKLOADS[args.workload]
    print(f"bench: generating {args.workload}", file=sys.stderr, flush=True)
    w = getattr(workloads, gen)()
    al = binding.Aligner(0)
    forms = ["batched", "plain"] if args.form == "both" else [args.form]
    if "batched" in forms:
        al.autotune(args.tune_cache)
    print(f"bench: timing {args.workload} ({', '.join(forms)})", file=sys.stderr, flush=True)
    legs = align_legs(args, al, w, forms, scoring, args.score_only, args.full_window)
    main_form = headline if headline in legs else forms[0]
    s, k, d = legs[main_form]
    if args.score_only:
        ops_model = f"{OPS_PER_CELL_SCORE} per window cell"
    elif args.full_window:
        ops_model = f"{OPS_PER_CELL} per window cell"
    else:
        ops_model = (f"{OPS_PER_CELL_SCORE} per window cell (score pass) + {OPS_PER_CELL} per "
                     f"band cell (decision pass)")
    line = {
        "metric": METRIC if not args.score_only else "GCUPS score only (no traceback), batched vs plain kernel",
        "value": round(w.cells / s / 1e9, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32" if main_form == "plain" else "int16+int32",
        "data": "synthetic",
        "config": {"workload": desc, "form": main_form, "n_tasks": w.n_tasks, "cells": w.cells,
                   "scoring": list(scoring)},
        "roofline": {
            "bound": "alu",
            "achieved": d["achieved_tops"],
            "peak": round(d["peak_tops"], 1),
            "unit": "TOP/s",
            "frac": d["valu_frac"],
            "traffic": None if args.score_only or args.full_window or args.score_scale != 1
                       else traffic_bytes(args.workload, main_form, d.get("shapes")),
            "ops_model": ops_model,
            "kernel_ms": d["device_ms"],
        },
        "forms": {f: v[2] for f, v in legs.items()},
    }
    default_run = not (args.score_only or args.full_window or args.score_scale != 1)
    issue = valu_issue_frac(args.workload, main_form, d["device_ms"], d.get("shapes"))
    if issue is not None and default_run:
        line["roofline"]["valu_issue_frac"] = issue
    for f in legs:
        fi = valu_issue_frac(args.workload, f, legs[f][2]["device_ms"], legs[f][2].get("shapes"))
        if fi is not None and default_run:
            line["forms"][f]["valu_issue_frac"] = fi
        tf = traffic_bytes(args.workload, f, legs[f][2].get("shapes"))
        if tf is not None and default_run:
            line["forms"][f]["traffic"] = tf
    if args.workload == "config5" and not args.no_extra and default_run:
        del w
        print("bench: generating config3", file=sys.stderr, flush=True)
        w3 = workloads.config3()
        print("bench: timing config3", file=sys.stderr, flush=True)
        legs3 = align_legs(args, al, w3, forms, scoring)
        line["uneven"] = {"workload": WORKLOADS["config3"][0], "cells": w3.cells,
                          "forms": {f: v[2] for f, v in legs3.items()}}
        del w3
        al.close()
        al = None
        torch.cuda.empty_cache()
        print(f"bench: served leg at {SERVE_QPS:.0f} requests/s", file=sys.stderr, flush=True)
        sv = serve_run(args, SERVE_QPS)
        line["served"] = {"workload": sv["config"]["workload"], "qps": SERVE_QPS,
                          "gcups": sv["value"], "latency_ms": sv["latency_ms"],
                          "latency_phases_ms": sv["latency_phases_ms"],
                          "slowest_launches": sv["slowest_launches"],
                          "achieved_qps": sv["achieved_qps"],
                          "slots": sv["config"]["slots"], "slot_tasks": sv["config"]["slot_tasks"],
                          "requests": sv["steps"],
                          "oracle_checked_requests": sv["oracle_checked_requests"]}
        line["latency_ms"] = {"p50": sv["latency_ms"]["p50"], "p99": sv["latency_ms"]["p99"],
                              "qps": SERVE_QPS}
        w = getattr(workloads, gen)()
    if not args.no_cpu_baseline:
        print("bench: oracle sample on the host", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_tasks, scoring)
    print(json.dumps(line), flush=True)
    if al is not None:
        al.close()


if __name__ == "__main__":
    main()
