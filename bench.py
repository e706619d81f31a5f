"""Benchmark of the split step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2|c5|c1]
                    [--precision fp64|fp32] [--no-cpu] [--profile]

Workload (default): the 2400 x 1800 spherical grid at 1 arc-minute
(seeded synthetic coast, shelf, slope and dipole source; 50 gauges; maxwave
every step), FP64.  A step is one full split step (x-sweep of every row,
y-sweep of every column, wet/dry cycle, maxwave, gauge records) of the
whole grid with the state resident in HBM.  Prints ONE JSON line.

value = cell-updates/s = nx * ny * K / (time of K steps), timed with HIP
events on the library's stream, bracketed by device synchronisation.

roofline: the fused step kernel alone (no gauges) is timed over K launches
with HIP events on its stream; achieved = algorithmic bytes per launch /
mean launch time, where one cell-step moves 11 words (read h, u, v, d;
write h, u, v; read and write the two maxwave arrays): 88 B in FP64,
44 B in FP32.  peak = 8 TB/s.

cpu_baseline: the FP64 oracle (OpenMP over rows / columns) on this host,
on a bounded sample of the same workload (a few full steps).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "split-step cell-updates/s (FP64, FP32) + % HBM roofline; ensemble and adjoint speedup"
PEAK_HBM = 8.0e12
WORDS_PER_CELL_STEP = 11


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_case(name, steps):
    from paper_1410_0753_amd import synth
    if name == "c2":
        return synth.config2(steps=steps)
    if name == "c5":
        return synth.config5(steps=steps)
    if name == "c1":
        return synth.config1(steps=steps)
    raise SystemExit("unknown workload " + name)


def time_steps(solver, torch, k):
    stream = solver.stream
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    solver.step(k)
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    solver.sync()
    return e0.elapsed_time(e1) / 1e3


def cpu_baseline(case, budget_s=12.0):
    import oracle
    o = oracle.Oracle.from_case(case)
    o.set_initial(case.eta0, case.u0, case.v0)
    t0 = time.perf_counter()
    o.step(1)
    t1 = time.perf_counter()
    per = t1 - t0
    k = max(1, min(200, int(budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    o.step(k)
    t1 = time.perf_counter()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": case.cells * k / (t1 - t0), "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d full FP64 split steps of the same %dx%d grid (after 1 warm-up step), "
                      "%.1f s" % (k, case.nx, case.ny, t1 - t0)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile", action="store_true", help="short run for profilers")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(every run here uses exactly one MI355X)", file=sys.stderr)
        sys.exit(2)
    if args.profile:
        args.steps, args.warmup, args.no_cpu = min(args.steps, 20), min(args.warmup, 3), True

    import numpy as np
    import torch
    from paper_1410_0753_amd import clf

    prec = clf.FP32 if args.precision == "fp32" else clf.FP64
    esize = 4 if prec == clf.FP32 else 8
    log("generating workload", args.workload)
    case = make_case(args.workload, args.steps)
    log("grid %dx%d dt %.4f" % (case.nx, case.ny, case.dt))
    torch.cuda.set_device(0)

    if args.calibrate_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # --- whole step: fused kernel + gauge records ---
    s = clf.Solver.from_case(case, precision=prec, gout=10, maxout=1, autotune=1,
                             gauge_capacity=(args.steps + args.warmup) // 10 + 8)
    s.set_initial(case.eta0, case.u0, case.v0)
    if case.gauges is not None:
        s.set_gauges(case.gauges[:, 0], case.gauges[:, 1])
    seg = int(s.query(clf.Q_SEGMENT))
    log("init done; segment %d rows, %d tiles" % (seg, s.query(clf.Q_TILES)))
    s.step(args.warmup)
    s.sync()
    secs = time_steps(s, torch, args.steps)
    value = case.cells * args.steps / secs
    log("step: %.3f ms, %.3e cell-updates/s" % (secs / args.steps * 1e3, value))
    e, _, _, w = s.state()
    log("max|eta| %.3f m, wet %d" % (float(e.abs().max()), int(w.sum())))
    del s

    # --- roofline leg: the step kernel alone ---
    r = clf.Solver.from_case(case, precision=prec, maxout=1, autotune=1)
    r.set_initial(case.eta0, case.u0, case.v0)
    r.step(args.warmup)
    r.sync()
    ksecs = time_steps(r, torch, args.steps)
    per_launch = ksecs / args.steps
    bytes_per_launch = WORDS_PER_CELL_STEP * esize * case.cells
    achieved = bytes_per_launch / per_launch
    del r

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == clf.FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": case.name + (" (%s, 50 gauges every 10 steps, maxwave every step)"
                                             % args.precision),
                   "nx": case.nx, "ny": case.ny, "dt": case.dt},
        "roofline": {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM, "traffic": None,
                     "kernel": "step_kernel (fused x-y march), %d B/cell-step algorithmic, "
                               "segment %d rows" % (WORDS_PER_CELL_STEP * esize, seg),
                     "mean_launch_ms": per_launch * 1e3},
    }
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
