"""Benchmark: GCUPS with traceback of the batched read-vs-window affine-gap
alignment on one MI355X, on the mate-rescue workload (1,000,000 reads x 100 bp
against 250 bp windows; seeded synthetic data).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--form plain|batched]

A step is one soap_dp_align_batch call over the whole batch (fill, traceback
and CIGAR for every task), inputs already resident in device memory.  Prints
one JSON line.
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
PEAK_INT32_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # CUs x SIMDs x lanes x clock = 39.3 T lane-ops/s
PEAK_INT16_TOPS = 2 * PEAK_INT32_TOPS            # packed 2 x int16 per lane


def cpu_baseline(w, tasks: int):
    import oracle
    idx = np.arange(min(tasks, w.n_tasks))
    cells = int(np.dot(w.read_len[idx].astype(np.int64), w.ref_len[idx].astype(np.int64)))
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    oracle.align_workload(w, oracle.scoring(*SCORING), idx=idx, n_threads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(cells / dt / 1e9, 4), "unit": "GCUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"first {idx.size:,} tasks of the same workload ({cells:.3g} cells), "
                      f"three-table int32 C oracle with traceback, {threads} threads, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", choices=["plain", "batched"], default="plain")
    ap.add_argument("--cpu-tasks", type=int, default=1_000_000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run device-to-device copies of BYTES (HBM counter calibration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; the tasks are independent and would be "
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
    w = workloads.config2()
    al = binding.Aligner(0)
    dw = binding.DeviceWorkload(w)
    res = binding.DeviceResult(w.n_tasks, 2 * dw.max_n)
    flags = binding.PLAIN if args.form == "plain" else binding.BATCHED
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        al.align(dw, SCORING, flags=flags, res=res)
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        al.align(dw, SCORING, flags=flags, res=res)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launch_ms = [a.elapsed_time(b) for a, b in ev]

    out = res.to_host()
    assert (out["status"] == 0).all(), "bench run produced invalid tasks"

    ms_per_step = elapsed * 1e3 / args.steps
    gcups = w.cells / (ms_per_step * 1e-3) / 1e9
    kern_ms = float(np.mean(launch_ms))
    achieved = OPS_PER_CELL * w.cells / (kern_ms * 1e-3) / 1e12
    peak = PEAK_INT32_TOPS if args.form == "plain" else PEAK_INT16_TOPS
    line = {
        "metric": METRIC,
        "value": round(gcups, 2),
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32" if args.form == "plain" else "int16+int32",
        "data": "synthetic",
        "config": {
            "workload": "mate-rescue: 1,000,000 reads x 100 bp vs 250 bp windows from a 1 Mbp "
                        "random genome (2% subs, 0.5% indels, 10% random reads)",
            "form": args.form,
            "n_tasks": w.n_tasks,
            "cells": w.cells,
            "scoring": list(SCORING),
        },
        "roofline": {
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": round(peak, 1),
            "unit": "TOP/s",
            "frac": round(achieved / peak, 4),
            "traffic": None,
            "ops_per_cell": OPS_PER_CELL,
            "kernel_ms": round(kern_ms, 3),
        },
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_tasks)
    print(json.dumps(line), flush=True)
    al.close()


if __name__ == "__main__":
    main()
