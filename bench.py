"""Benchmark: GCUPS with traceback of batched read-vs-window affine-gap
alignment on one MI355X (seeded synthetic data).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload config2|config3|config5|config4|multi|mate]

Default workload: the mate-rescue batch, 1,000,000 reads x 100 bp against
250 bp windows, aligned by the plain one-launch int32 kernel (`value`); the
batched form (length classes, packed int16 with int32 re-run, persistent
kernels, graph replay, autotuned shapes) runs on the same data and is
reported beside it.  A step is one soap_dp_align_batch call over the whole
batch (fill, traceback and CIGAR of every task), inputs resident in device
memory.  Prints one JSON line.
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
PEAK_INT32_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # CUs x SIMDs x lanes x clock = 39.3 T lane-ops/s
PEAK_INT16_TOPS = 2 * PEAK_INT32_TOPS            # packed 2 x int16 per lane

# HBM traffic of the dominant kernel per launch, from two rocprofv3 --pmc
# runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) scaled by what the same
# counters read for a plain 1 GiB device copy (FETCH x 2.000, WRITE x 1.000).
# Keyed by (workload, form); valid only for the kernel sources fingerprinted
# (any change to them makes `traffic` null until the counters are re-taken).
KERNEL_SOURCES = ("api.cpp", "batch.h", "batch.hip", "dp_device.h", "dp_i16.hip", "dp_i32.hip",
                  "dp_internal.h")
TRAFFIC = {
    ("config2", "plain"): {"fingerprint": "574b7377cdc0bf7b", "kernel": "dp_i32_kernel<4,25,byte>",
                           "fetch_kib": 2456014, "write_kib": 16142110,
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


def traffic_bytes(workload: str, form: str):
    t = TRAFFIC.get((workload, form))
    if t is None or t["fingerprint"] != kernel_fingerprint():
        return None
    return int(round((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024))


WORKLOADS = {
    "config2": ("mate-rescue: 1,000,000 reads x 100 bp vs 250 bp windows from a 1 Mbp random "
                "genome (2% subs, 0.5% indels, 10% random reads)", "config2", "plain"),
    "config3": ("uneven: 2,000,000 reads, n uniform over {36,50,75,100,150,250}, m = n + 160 "
                "(4% subs, 0.5% indels up to 30 bp)", "config3", "batched"),
    "config5": ("low-similarity: 500,000 reads x 150 bp at 60-75% identity vs 1,000 bp windows",
                "config5", "batched"),
}


def cpu_baseline(w, tasks: int):
    import oracle
    idx = np.arange(min(tasks, w.n_tasks))
    cells = int(np.dot(w.read_len[idx].astype(np.int64), w.ref_len[idx].astype(np.int64)))
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    oracle.align_workload(w, oracle.scoring(*SCORING), idx=idx, n_threads=threads)
    dt = time.perf_counter() - t0
    what = "all" if idx.size == w.n_tasks else f"first {idx.size:,}"
    # one core on a fixed 20,000-task prefix
    idx1 = np.arange(min(20_000, w.n_tasks))
    cells1 = int(np.dot(w.read_len[idx1].astype(np.int64), w.ref_len[idx1].astype(np.int64)))
    t1 = time.perf_counter()
    oracle.align_workload(w, oracle.scoring(*SCORING), idx=idx1, n_threads=1)
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
    """Served workload: Poisson arrivals of requests of 1..4096 reads
    (log-uniform), reads 50-250 bp over a device-resident 100 Mbp genome.
    With --qps 0 the requests all arrive at once, which measures capacity."""
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
                         autotune=True, device_bytes=args.device_bytes)
    qps = args.qps if args.qps is not None else SERVE_QPS
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
                   "slot_tasks": args.slot_tasks,
                   "requests": args.serve_requests, "mean_cells_per_request": round(mean_cells)},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3),
                       "max": round(float(lat.max()), 3)},
        "latency_phases_ms": breakdown,
        "achieved_qps": round((args.serve_requests if qps > 0 else n_total) / span, 1),
        "late_submissions": int((lag[meas] > 0).sum()),
        "server": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in st.items()},
        "oracle_checked_requests": checked,
    }
    print(json.dumps(line), flush=True)


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


def time_form(al, dw, res, flags, steps, warmup):
    import torch
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        al.align(dw, SCORING, flags=flags, res=res)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        al.align(dw, SCORING, flags=flags, res=res)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    out = res.to_host()
    assert (out["status"] != 1).all() and (out["status"] != 3).all(), "invalid tasks in bench"
    time_form.redone = float(np.mean(out["status"] == 2))
    return elapsed / steps, float(np.mean([a.elapsed_time(b) for a, b in ev]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["config4", "multi", "mate"],
                    default="config2")
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
    ap.add_argument("--serve-warmup", type=int, default=1000)
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--form", choices=["plain", "batched", "both"], default="both")
    ap.add_argument("--cpu-tasks", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--score-only", action="store_true",
                    help="score and end only (SOAP_DP_SCORE_ONLY), no traceback")
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
    global SCORING
    if args.score_scale != 1:
        SCORING = tuple(args.score_scale * x for x in SCORING)
    desc, gen, headline = WORKLOADS[args.workload]
    w = getattr(workloads, gen)()
    al = binding.Aligner(0)
    dw = binding.DeviceWorkload(w)
    # --score-only: score and end of every task, no traceback (its own
    # kernels and shapes); reported at 10 ops per cell
    extra = binding.SCORE_ONLY if args.score_only else 0
    ops = OPS_PER_CELL_SCORE if args.score_only else OPS_PER_CELL
    res = binding.DeviceResult(w.n_tasks, 0 if args.score_only else 2 * dw.max_n)

    forms = {}
    if args.form in ("batched", "both"):
        al.autotune(args.tune_cache)
        s, k = time_form(al, dw, res, binding.BATCHED | extra, args.steps, args.warmup)
        forms["batched"] = (s, k)
        redone = time_form.redone
    if args.form in ("plain", "both"):
        s, k = time_form(al, dw, res, binding.PLAIN | extra, args.steps, args.warmup)
        forms["plain"] = (s, k)
    main_form = headline if headline in forms else next(iter(forms))

    def summary(form):
        s, k = forms[form]
        peak = PEAK_INT32_TOPS if form == "plain" else PEAK_INT16_TOPS
        achieved = ops * w.cells / (k * 1e-3) / 1e12
        return s, k, peak, achieved

    s, k, peak, achieved = summary(main_form)
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
                   "scoring": list(SCORING)},
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": round(peak, 1),
            "unit": "TOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": None if args.score_only else traffic_bytes(args.workload, main_form),
            "ops_per_cell": ops,
            "kernel_ms": round(k, 3),
        },
        "forms": {},
    }
    for form in forms:
        fs, fk, fpeak, fach = summary(form)
        line["forms"][form] = {"gcups": round(w.cells / fs / 1e9, 2), "ms_per_step": round(fs * 1e3, 3),
                               "device_ms": round(fk, 3), "valu_frac": round(fach / fpeak, 4),
                               "peak_tops": round(fpeak, 1)}
    if "batched" in forms:
        lengths = sorted(set(int(x) for x in np.unique(w.read_len)))
        shapes = {}
        for prec, cap, lanes, cells in al.classes():
            hit = [n for n in lengths if n <= cap and not any(n <= c for p2, c, _, _ in al.classes()
                                                                if p2 == prec and c < cap)]
            if prec == 16 and hit:
                shapes[str(cap)] = f"{lanes}x{cells}"
        line["forms"]["batched"]["shapes"] = shapes
        line["forms"]["batched"]["redone_int32"] = round(redone, 4)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_tasks)
    print(json.dumps(line), flush=True)
    al.close()


if __name__ == "__main__":
    main()
