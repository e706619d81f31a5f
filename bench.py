"""Benchmark of the split step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--workload c2|c5|c1|ensemble|adjoint|c5err]
                    [--precision fp64|fp32] [--no-cpu] [--no-extras] [--profile]

Headline (default): the 2400 x 1800 spherical grid at 1 arc-minute (seeded
synthetic coast, shelf, slope and dipole source; 50 gauges every 10 steps;
maxwave every step) in FP64.  A step is one full split step (x-sweep of every
row, y-sweep of every column, wet/dry cycle, maxwave, gauge records) of the
whole grid with the state resident in HBM.  Prints ONE JSON line.

value = cell-updates/s = nx * ny * K / (time of K steps), timed with HIP
events on the library's stream, bracketed by device synchronisation.

roofline: the fused step kernel alone is timed over K launches with HIP
events on its stream; achieved = algorithmic bytes per launch / mean launch
time, where one cell-step moves 11 words (read h, u, v, d; write h, u, v;
read and write the two maxwave arrays): 88 B in FP64, 44 B in FP32.
peak = 8 TB/s; copy_GBps is a measured 1 GiB device copy on the same GPU
(what a plain streaming kernel attains).  `traffic` is the calibrated
rocprofv3 FETCH_SIZE + WRITE_SIZE of the kernel per launch when the kernel
source is the one that was profiled (else null).

cpu_baseline: the FP64 oracle (OpenMP over rows / columns) on this host, on
a bounded number of full steps of the same grid, plus a shorter
single-thread sample.

extras (same line): the FP32 run of the headline grid with its error
against the FP64 oracle; the 8000 x 6000 spherical grid (FP32 and FP64, with
its 4 enclosed-grid boundary series every step); the 64-member
ensemble against sequential single-grid solves; the adjoint gradient of the
1000 x 800 inversion problem against a finite-difference gradient (and an
estimate of the same gradient by the host oracle); the oracle's rate on the
200 x 200 and 8000 x 6000 grids.

--workload c5err (not part of the default run) reports the FP32 error on the
8000 x 6000 grid: against the FP64 oracle after min(K, 50) steps and against
the FP64 GPU path after K steps.
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

METRIC = "split-step cell-updates/s (FP64, FP32) + % HBM roofline; ensemble and adjoint speedup"
PEAK_HBM = 8.0e12
WORDS_PER_CELL_STEP = 11
KERNEL_SRC = os.path.join(ROOT, "paper_1410_0753_amd", "csrc", "clf_kernels.hip")
# Calibrated HBM bytes per launch of the step kernel, from rocprofv3 --pmc
# FETCH_SIZE / WRITE_SIZE runs (profiles/), keyed by the sha256 of the kernel
# source they were taken on and by workload, one entry per measured launch
# shape; an entry applies only to a launch of the same workgroup count
# (segment length), which the autotuner may choose differently run to run.
TRAFFIC = {
    "9c29862b1b599625c1c0a3659d6523945f28be11f0b9c419852ef46673b71221": {
        "c2/fp64": [{"workgroups": 760, "read_bytes": 236000000, "write_bytes": 111200000}],
        "c2/fp32": [{"workgroups": 1000, "read_bytes": 115900000, "write_bytes": 52700000}],
        "c5/fp32": [{"workgroups": 4072, "read_bytes": 1314500000, "write_bytes": 604300000},
                    {"workgroups": 4320, "read_bytes": 1324600000, "write_bytes": 601600000}],
        "c5/fp64": [{"workgroups": 3072, "read_bytes": 2555100000, "write_bytes": 1218600000},
                    {"workgroups": 2280, "read_bytes": 2554200000, "write_bytes": 1225700000}],
    },
}


def traffic_entry(sha, key, workgroups):
    """The calibrated traffic of a launch of `workgroups` workgroups of the
    kernel source `sha` on workload `key`, or None when it was not measured
    (another source, workload or launch shape)."""
    return next((t for t in TRAFFIC.get(sha, {}).get(key, [])
                 if t["workgroups"] == workgroups), None)


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


def kernel_sha():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()


def timed(torch, stream, fn):
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn()
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def run_grid(case, prec, steps, warmup, gauges=True, enclosed=False, bndout=1):
    """Whole-step throughput (with gauges, and the enclosed-grid boundary
    series every `bndout` steps when `enclosed`) and the step kernel alone."""
    import torch
    from paper_1410_0753_amd import clf
    esize = 4 if prec == clf.FP32 else 8
    kw = {}
    if enclosed and case.enclosed:
        kw = dict(bndout=bndout, max_enclosed=len(case.enclosed),
                  series_capacity=(steps + warmup) // bndout + 8)
    s = clf.Solver.from_case(case, precision=prec, gout=10, maxout=1, autotune=1,
                             gauge_capacity=(steps + warmup) // 10 + 8, **kw)
    s.set_initial(case.eta0, case.u0, case.v0)
    if gauges and case.gauges is not None:
        s.set_gauges(case.gauges[:, 0], case.gauges[:, 1])
    if kw:
        for ex, ey in case.enclosed:
            s.add_enclosed_grid(ex, ey)
    dry0 = s.state()[3] == 0
    seg = int(s.query(clf.Q_SEGMENT))
    s.step(warmup)
    s.sync()
    secs = timed(torch, s.stream, lambda: s.step(steps))
    s.sync()
    e, _, _, w = s.state()
    emax = s.read_maxwave()[0]
    ever_wet = float(((emax > 0) & dry0).sum()) / max(1.0, float(dry0.sum()))
    log("%s %s: %.4f ms/step, segment %d, max|eta| %.3f, wet %d" % (
        case.name, "fp32" if prec == clf.FP32 else "fp64", secs / steps * 1e3, seg,
        float(e.abs().max()), int(w.sum())))
    del s
    r = clf.Solver.from_case(case, precision=prec, maxout=1, autotune=1, graph_steps=0)
    r.set_initial(case.eta0, case.u0, case.v0)
    r.step(warmup)
    r.sync()
    ksecs = timed(torch, r.stream, lambda: r.step(steps))
    r.sync()
    per_launch = ksecs / steps
    achieved = WORDS_PER_CELL_STEP * esize * case.cells / per_launch
    blocks = int(r.query(clf.Q_BLOCKS))
    del r
    return {"value": case.cells * steps / secs, "ms_per_step": secs / steps * 1e3,
            "segment": seg, "kernel_ms": per_launch * 1e3, "achieved": achieved,
            "workgroups": blocks,
            "ever_wet_frac_of_initially_dry": ever_wet,
            "enclosed_grids": len(case.enclosed) if kw else 0}


def copy_bandwidth():
    """Device-to-device copy of 1 GiB (read + write bytes / time): the
    attainable HBM rate of a plain streaming kernel on this GPU."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    reps = 10
    stream = torch.cuda.current_stream()
    secs = timed(torch, stream, lambda: [b.copy_(a) for _ in range(reps)])
    del a, b
    return 2.0 * (1 << 30) * reps / secs


def fp32_error(case, steps):
    """FP32 GPU vs FP64 oracle after `steps` steps: max/RMS eta error over the
    amplitude, fraction of nodes whose wet flag differs."""
    import numpy as np
    import oracle
    from paper_1410_0753_amd import clf
    g = clf.Solver.from_case(case, precision=clf.FP32)
    o = oracle.Oracle.from_case(case)
    for obj in (g, o):
        obj.set_initial(case.eta0, case.u0, case.v0)
        obj.step(steps)
    eg, _, _, wg = (t.cpu().numpy() for t in g.state())
    eo, _, _, wo = o.state()
    amp = float(np.abs(eo).max())
    err = np.abs(eg - eo)
    return {"steps": steps, "max_eta_err_rel": float(err.max() / amp),
            "rms_eta_err_rel": float(np.sqrt((err ** 2).mean()) / amp),
            "mask_flip_frac": float((wg.astype(bool) != wo.astype(bool)).mean())}


def run_ensemble(steps, n=64):
    import torch
    from paper_1410_0753_amd import clf, synth
    log("generating %d ensemble members" % n)
    cases = synth.config3(n=n, steps=steps)
    cells = sum(c.cells for c in cases)
    ens = clf.Ensemble(cases, precision=clf.FP32, maxout=1, autotune=1)
    for i, c in enumerate(cases):
        ens.set_initial(i, c.eta0, c.u0, c.v0)
    ens.step(16)
    ens.sync()
    tb = timed(torch, ens.stream, lambda: ens.step(steps))
    ens.sync()
    seg, blocks = int(ens.query(clf.Q_SEGMENT)), int(ens.query(clf.Q_BLOCKS))
    del ens
    # sequential single-grid solves (each autotuned, same precision and steps)
    solvers = []
    for c in cases:
        s = clf.Solver.from_case(c, precision=clf.FP32, maxout=1, autotune=1)
        s.set_initial(c.eta0, c.u0, c.v0)
        s.step(16)
        solvers.append(s)
    torch.cuda.synchronize()

    def seq():
        for s in solvers:
            s.step(steps)

    ts = timed(torch, solvers[0].stream, seq)
    del solvers
    return {"members": n, "cells": cells, "steps": steps, "precision": "fp32",
            "batched_cell_updates_per_s": cells * steps / tb,
            "sequential_cell_updates_per_s": cells * steps / ts,
            "speedup_vs_sequential": ts / tb, "segment": seg, "workgroups": blocks,
            "roofline_frac": cells * steps / tb * WORDS_PER_CELL_STEP * 4 / PEAK_HBM}


def run_adjoint(steps=3000, cpu_fd=False):
    import numpy as np
    import torch
    from paper_1410_0753_amd import clf, synth
    case, basis, c_true, c0 = synth.config4(steps=steps)
    s = clf.Solver.from_case(case, gout=1, gauge_capacity=steps + 2)
    s.set_gauges(case.gauges[:, 0], case.gauges[:, 1])
    B = torch.tensor(basis, device="cuda")

    def eta(c):
        return torch.tensordot(torch.tensor(c, device="cuda"), B, dims=1)

    s.set_initial(eta(c_true))
    s.step(steps)
    obs = s.read_gauges()[0][:, :, 0].copy()

    def loss(c):
        s.set_initial(eta(c))
        s.step(steps)
        rec = s.read_gauges()[0][:, :, 0]
        return 0.5 * float(np.sum((rec - obs) ** 2))

    loss(c0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.set_initial(eta(c0))
    s.adjoint_forward(steps, 0)
    rec = s.read_gauges()[0]
    adj = np.zeros_like(rec)
    adj[:, :, 0] = rec[:, :, 0] - obs
    g_eta = s.adjoint_backward(adj)[0]
    g = torch.tensordot(B, g_eta, dims=([1, 2], [0, 1])).cpu().numpy()
    t_adj = time.perf_counter() - t0
    h = 1e-4
    t0 = time.perf_counter()
    fd = np.zeros_like(c0)
    for k in range(len(c0)):
        e = np.zeros_like(c0)
        e[k] = h
        fd[k] = (loss(c0 + e) - loss(c0 - e)) / (2 * h)
    t_fd = time.perf_counter() - t0
    rel = float(np.max(np.abs(g - fd)) / np.max(np.abs(fd)))
    extra = {}
    if cpu_fd:
        # the same finite-difference gradient on the host oracle, estimated
        # from a timed 50-step forward solve with the gauges recorded
        import oracle
        o = oracle.Oracle.from_case(case, gout=1)
        o.set_gauges(case.gauges[:, 0], case.gauges[:, 1])
        o.set_initial(case.eta0)
        t0 = time.perf_counter()
        o.step(50)
        per = (time.perf_counter() - t0) / 50
        extra = {"cpu_oracle_fd_s_estimate": 2 * len(c0) * steps * per,
                 "cpu_oracle_fd_basis": "50-step oracle sample on %d threads, scaled to %d solves "
                                        "of %d steps" % (oracle.set_threads(0), 2 * len(c0), steps)}
        extra["speedup_vs_cpu_oracle_fd"] = extra["cpu_oracle_fd_s_estimate"] / t_adj
        del o
    return {**extra, "grid": "%dx%d" % (case.nx, case.ny), "steps": steps, "sources": len(c0),
            "gauges": int(len(case.gauges)), "checkpoint_every": int(np.ceil(np.sqrt(steps))),
            "adjoint_s": t_adj, "fd_s": t_fd, "speedup_vs_fd": t_fd / t_adj,
            "max_rel_diff_vs_fd": rel}


def cpu_baseline(case, budget_s=12.0):
    import oracle
    o = oracle.Oracle.from_case(case)
    o.set_initial(case.eta0, case.u0, case.v0)
    t0 = time.perf_counter()
    o.step(1)
    per = time.perf_counter() - t0
    k = max(1, min(200, int(budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    o.step(k)
    t1 = time.perf_counter()
    threads = oracle.set_threads(0)
    # the same oracle on one thread, a shorter sample
    oracle.set_threads(1)
    k1 = max(1, min(k, int(0.25 * budget_s / max(per * threads, 1e-6))))
    t2 = time.perf_counter()
    o.step(k1)
    t3 = time.perf_counter()
    oracle.set_threads(threads)
    return {"value": case.cells * k / (t1 - t0), "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": "%d full FP64 split steps of the same %dx%d grid (after 1 warm-up step), "
                      "%.1f s" % (k, case.nx, case.ny, t1 - t0),
            "single_thread_value": case.cells * k1 / (t3 - t2),
            "single_thread_sample": "%d further steps on 1 thread, %.1f s" % (k1, t3 - t2)}


def cpu_other(cases):
    """The oracle on other workloads: steps per second on a few full steps
    (after one warm-up step), all host threads."""
    import oracle
    out = {}
    for name, case, k in cases:
        o = oracle.Oracle.from_case(case)
        o.set_initial(case.eta0, case.u0, case.v0)
        o.step(1)
        t0 = time.perf_counter()
        o.step(k)
        dt = time.perf_counter() - t0
        out[name] = {"cell_updates_per_s": case.cells * k / dt, "steps": k,
                     "grid": "%dx%d" % (case.nx, case.ny), "seconds": dt}
        del o
    out["cores"] = oracle.set_threads(0)
    return out


def fp32_error_large(steps, oracle_steps):
    """FP32 on the 8000x6000 grid against the FP64 oracle after
    `oracle_steps` steps, and against the FP64 GPU path (bitwise equal to the
    oracle on every parity test) after `steps` steps."""
    import numpy as np
    import oracle
    from paper_1410_0753_amd import clf, synth
    case = synth.config5(steps=steps)

    def run(prec, n):
        s = clf.Solver.from_case(case, precision=prec, maxout=1, autotune=1)
        s.set_initial(case.eta0, case.u0, case.v0)
        dry0 = (s.state()[3] == 0).cpu().numpy()
        s.step(n)
        e, _, _, w = (t.cpu().numpy() for t in s.state())
        em = s.read_maxwave()[0].cpu().numpy()
        del s
        return e, w, em, dry0

    def compare(ea, wa, eb, wb):
        amp = float(np.abs(eb).max())
        err = np.abs(ea - eb)
        return {"max_eta_err_rel": float(err.max() / amp),
                "rms_eta_err_rel": float(np.sqrt((err ** 2).mean()) / amp),
                "mask_flip_frac": float((wa.astype(bool) != wb.astype(bool)).mean())}

    log("fp32 vs oracle, %d steps ..." % oracle_steps)
    e32, w32, _, _ = run(clf.FP32, oracle_steps)
    o = oracle.Oracle.from_case(case)
    o.set_initial(case.eta0, case.u0, case.v0)
    t0 = time.perf_counter()
    o.step(oracle_steps)
    to = time.perf_counter() - t0
    eo, _, _, wo = o.state()
    del o
    res = {"workload": case.name, "vs_fp64_oracle": dict(steps=oracle_steps, oracle_s=to,
                                                         **compare(e32, w32, eo, wo))}
    log("fp32 vs fp64 gpu, %d steps ..." % steps)
    e32, w32, m32, dry0 = run(clf.FP32, steps)
    e64, w64, m64, _ = run(clf.FP64, steps)
    ew32, ew64 = (m32 > 0) & dry0, (m64 > 0) & dry0
    res["vs_fp64_gpu"] = dict(steps=steps, **compare(e32, w32, e64, w64))
    res["vs_fp64_gpu"]["ever_wet_of_initially_dry_fp32"] = float(ew32.sum() / max(1, dry0.sum()))
    res["vs_fp64_gpu"]["ever_wet_of_initially_dry_fp64"] = float(ew64.sum() / max(1, dry0.sum()))
    res["vs_fp64_gpu"]["ever_wet_flip_frac"] = float((ew32 != ew64).mean())
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--profile", action="store_true", help="short run for profilers")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(the y-band sharding design is described but not built); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if args.profile:
        args.steps, args.warmup = min(args.steps, 20), min(args.warmup, 3)
        args.no_cpu = args.no_extras = True

    import torch
    from paper_1410_0753_amd import clf

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.workload == "c5err":
        # long-run FP32 error report on the 8000x6000 grid (not in the default run)
        res = fp32_error_large(args.steps, min(args.steps, 50))
        print(json.dumps({"metric": METRIC, "workload": "c5err", "fp32_error": res}), flush=True)
        return
    if args.workload in ("ensemble", "adjoint"):
        # one extras leg alone (for profilers)
        torch.cuda.set_device(0)
        if args.workload == "ensemble":
            res = run_ensemble(20 if args.profile else min(args.steps, 300),
                               n=16 if args.profile else 64)
        else:
            res = run_adjoint(200 if args.profile else 3000)
        print(json.dumps({"metric": METRIC, "workload": args.workload, args.workload: res}),
              flush=True)
        return

    prec = clf.FP32 if args.precision == "fp32" else clf.FP64
    esize = 4 if prec == clf.FP32 else 8
    log("generating workload", args.workload)
    case = make_case(args.workload, args.steps)
    head = run_grid(case, prec, args.steps, args.warmup)
    copy_bw = None if args.profile else copy_bandwidth()
    traffic = None
    tr = traffic_entry(kernel_sha(), "%s/%s" % (args.workload, args.precision),
                       head["workgroups"])
    if tr:
        tb = tr["read_bytes"] + tr["write_bytes"]
        traffic = {"GBps": tb / (head["kernel_ms"] * 1e-3) / 1e9,
                   "bytes_per_launch": tb, "read_bytes": tr["read_bytes"],
                   "write_bytes": tr["write_bytes"],
                   "algorithmic_bytes_per_launch": WORDS_PER_CELL_STEP * esize * case.cells}
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == clf.FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": case.name + (" (%s, 50 gauges every 10 steps, maxwave every step)"
                                             % args.precision),
                   "nx": case.nx, "ny": case.ny, "dt": case.dt},
        "roofline": {"bound": "hbm", "achieved": head["achieved"] / 1e9,
                     "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                     "frac": head["achieved"] / PEAK_HBM, "traffic": traffic,
                     "kernel": "step_kernel (fused x-y march), %d B/cell-step algorithmic, "
                               "segment %d rows" % (WORDS_PER_CELL_STEP * esize, head["segment"]),
                     "mean_launch_ms": head["kernel_ms"],
                     "copy_GBps": copy_bw / 1e9 if copy_bw else None,
                     "frac_of_copy": head["achieved"] / copy_bw if copy_bw else None,
                     "frac_of_two_sweep_model": head["value"] * 18 * esize / PEAK_HBM,
                     "note": "frac uses the fused kernel's 11 words per cell-step; "
                             "frac_of_two_sweep_model the 18 words of two separate sweeps "
                             "with maxwave. Grids up to about 2400x1800 FP64 fit the 256 MB "
                             "Infinity Cache; the HBM-resident runs are the 8000x6000 extras."},
    }
    if not args.no_cpu:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(case)
    if not args.no_extras:
        from paper_1410_0753_amd import synth
        extras = {}
        if prec == clf.FP64:
            r32 = run_grid(case, clf.FP32, args.steps, args.warmup)
            r32["roofline_frac"] = r32.pop("achieved") / PEAK_HBM
            log("fp32 error vs oracle ...")
            r32["error_vs_fp64_oracle"] = fp32_error(case, 200)
            extras["fp32_same_grid"] = r32
        log("8000x6000 spherical grid ...")
        big = synth.config5(steps=args.steps)
        rb = run_grid(big, clf.FP32, min(args.steps, 400), 20, enclosed=True)
        rb["roofline_frac"] = rb.pop("achieved") / PEAK_HBM
        rb["workload"] = big.name + (" (fp32, 50 gauges every 10 steps, maxwave every step, "
                                     "4 enclosed-grid boundary series every step)")
        extras["large_grid_fp32"] = rb
        log("8000x6000 spherical grid, fp64 ...")
        rb = run_grid(big, clf.FP64, min(args.steps, 100), 10, enclosed=True)
        rb["roofline_frac"] = rb.pop("achieved") / PEAK_HBM
        rb["workload"] = big.name + (" (fp64, 50 gauges every 10 steps, maxwave every step, "
                                     "4 enclosed-grid boundary series every step)")
        extras["large_grid_fp64"] = rb
        if not args.no_cpu:
            log("oracle on the other workloads ...")
            extras["cpu_other"] = cpu_other([("200x200", synth.config1(steps=10), 400),
                                             ("8000x6000", big, 2)])
        del big
        log("ensemble ...")
        extras["ensemble"] = run_ensemble(min(args.steps, 300))
        log("adjoint ...")
        extras["adjoint"] = run_adjoint(3000, cpu_fd=not args.no_cpu)

        out["extras"] = extras
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
