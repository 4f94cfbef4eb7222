#!/usr/bin/env python3
"""Throughput of the fused VP-LBM step on one MI355X.

Workload: NACA 0012 (4-digit thickness form, chord 200 cells) at 10 degrees
angle of attack in a 2000 x 1000 channel (inflow 0.05, tau = 0.53, Re = 1000,
eta = 1e-4), 401 stress-integration points, FP32 deviation storage.  One
"step" is one full time step of the path: the fused stream / penalize /
collide / momentum-exchange / stress-integration kernel plus the force
finalize.  Inputs are resident in HBM before timing starts.

Prints one JSON line (metric, MLUPS value, roofline of the step kernel, CPU
oracle baseline).  Only one GPU is supported.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS and % HBM roofline per step; p50/p99 solve latency under mixed-size load"
HBM_PEAK_GBS = 8000.0
BYTES_PER_CELL = {"f64": 9 * 8 * 2 + 1, "f32": 9 * 4 * 2 + 1, "f16dev": 9 * 2 * 2 + 1}


COUNTERS = os.path.join(ROOT, "profiles", "k_step_naca0012_2000x1000_f32_hbm_counters.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2110_00967_amd", "csrc", f) for f in ("d2q9.hpp", "step_kernel.hpp")]


def measured_traffic():
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    summary, or None when the kernel source changed since it was taken."""
    import hashlib

    if not os.path.exists(COUNTERS):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    vals = {}
    with open(COUNTERS) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("#", "|", "`")):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if vals.get("kernel_source_sha256") != h.hexdigest():
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_baseline(case, budget_s=12.0):
    """The FP64 oracle on the host cores, on a bounded number of steps."""
    import oracle as O

    lat = O.RefLattice.from_case(case)
    lat.step(2)  # warm-up (page-in, thread pool)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s or n < 3:
        lat.step(1)
        n += 1
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": case.nx * case.ny * n / dt / 1e6,
        "unit": "MLUPS",
        "cores": min(threads, os.cpu_count() or 1),
        "kind": "oracle",
        "sample": f"{case.name} {case.nx}x{case.ny} FP64 oracle, {n} steps ({dt:.1f} s), "
                  f"OpenMP over rows, CPU {platform.processor() or platform.machine()}",
    }


def run_sweep(args, torch, W, V, paper=False):
    """Many airfoil cases stepped by one launch per step, and the same cases
    stepped one after the other (the plain single-case form).  Default: 64
    cases (chords 100/150/200, AoA 0-20 deg).  paper: the paper's full-scale
    runs, chord 278 on 3614 x 1946, TRT, AoA 0-28 deg in steps of 2."""
    cases = W.paper_aoa_sweep() if paper else W.sweep_cases()
    st = V.STREAM_AA if args.streaming == "aa" else V.STREAM_AB
    lats = [V.Lattice.from_case(c, precision=args.precision, streaming=st) for c in cases]
    cells = sum(c.nx * c.ny for c in cases)
    batch = V.Batch(lats)
    n = len(lats)
    batch.step([args.warmup] * n)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    batch.step([args.steps] * n)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # serial form: each case alone, one after the other, same number of steps
    ks = max(args.steps // 4, 1)
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    for lat in lats:
        lat.step(ks)
    s1.record()
    torch.cuda.synchronize()
    ms_serial = s0.elapsed_time(s1) / ks
    bpc = BYTES_PER_CELL[args.precision]
    achieved = bpc * cells / (ms * 1e-3) / 1e9
    q = [0.5 * c.u_ref ** 2 * c.length_scale for c in cases]
    cd = [lat.forces_si()[0] / qq for lat, qq in zip(lats, q)]
    if paper:
        config = {"workload": "naca0012_paper_c278_3614x1946_trt_aoa_sweep", "cases": n, "cells": cells,
                  "chord": 278, "aoa_deg": [0.0, 2.0 * (n - 1)],
                  "tau": 0.55, "trt_lambda": round(1.0 / 6.0, 6), "eta": 1e-6, "si_points": len(cases[0].si_ds),
                  "storage": args.precision, "streaming": args.streaming.upper(),
                  "parallelism": "single GPU, one batched launch per step"}
    else:
        config = {"workload": "naca0012_aoa_sweep_64cases", "cases": n, "cells": cells,
                  "chords": [100, 150, 200], "aoa_deg": [0.0, 20.0], "storage": args.precision,
                  "streaming": args.streaming.upper(), "parallelism": "single GPU, one batched launch per step"}
    out = {
        "metric": METRIC, "value": round(cells / (ms * 1e-3) / 1e6, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32", "f16dev": "f32 (f16 storage)", "f64": "f64"}[args.precision],
        "data": "synthetic",
        "config": config,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_step_batch",
                     "kernel_us": round(ms * 1e3, 3), "bytes_per_cell": bpc, "cells_per_launch": cells},
        "serial": {"ms_per_step": round(ms_serial, 5), "MLUPS": round(cells / (ms_serial * 1e-3) / 1e6, 1),
                   "steps": ks},
        "CD_SI_range": [round(min(cd), 4), round(max(cd), 4)],
    }
    if paper:
        # force coefficients after the run, per angle (both methods; the
        # paper's own curves are not available to compare with)
        out["coefficients"] = [
            {"aoa_deg": 2.0 * k, "CD_ME": round(lat.forces_me()[0] / qq, 5), "CL_ME": round(lat.forces_me()[1] / qq, 5),
             "CD_SI": round(lat.forces_si()[0] / qq, 5), "CL_SI": round(lat.forces_si()[1] / qq, 5)}
            for k, (lat, qq) in enumerate(zip(lats, q))]
        out["steps_run"] = lats[0].step_count
    batch.close()
    for lat in lats:
        lat.close()
    return out


def run_sed_paper(args, torch, W, V):
    """The paper's sedimentation runs at full scale: one free disk (D = 26,
    tau = 0.6, eta = 1e-6) per printed density ratio and per force source
    driving it (SI and ME, the paper's comparison), stepped together by one
    batched step launch and one batched body launch per step.
    --sed-seconds > 0 also runs the cases to that physical time and reports
    each disk's trajectory every 0.1 s."""
    cases = W.paper_sedimentation_sweep(force_source=1) + W.paper_sedimentation_sweep(force_source=0)
    st = V.STREAM_AA if args.streaming == "aa" else V.STREAM_AB
    lats = [V.Lattice.from_case(c, precision=args.precision, streaming=st) for c in cases]
    cells = sum(c.nx * c.ny for c in cases)
    batch = V.Batch(lats)
    n = len(lats)
    batch.step([args.warmup] * n)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    batch.step([args.steps] * n)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    _, dt, g = W.paper_sedimentation_units()
    nu = (0.6 - 0.5) / 3.0

    def state(c, lat):
        x, y, th, u, v, om = lat.body_state()
        return {"t_s": round(lat.step_count * dt, 4), "x_over_D": round((x + 0.5) / c.length_scale, 4),
                "fall_over_D": round((c.disk[1] - y) / c.length_scale, 4),
                "Re": round(math.hypot(u, v) * c.length_scale / nu, 4), "omega": om}

    traj = [[] for _ in cases]
    if args.sed_seconds > 0:
        # the rest of the run to the given physical time, sampled every 0.1 s
        total = int(round(args.sed_seconds / dt))
        every = int(round(0.1 / dt))
        while lats[0].step_count < total:
            k = min(every - lats[0].step_count % every, total - lats[0].step_count)
            batch.step([k] * n)
            torch.cuda.synchronize()
            if lats[0].step_count % every == 0:
                for t, c, lat in zip(traj, cases, lats):
                    t.append(state(c, lat))
                print(f"[sediment-paper] {lats[0].step_count} steps", file=sys.stderr, flush=True)
    bodies = []
    for c, lat, t in zip(cases, lats, traj):
        b = {"rho_r": c.rho_s, "source": "SI" if c.force_source == 1 else "ME", "steps": lat.step_count,
             **state(c, lat)}
        if t:
            b["trajectory"] = t
        bodies.append(b)
    bpc = BYTES_PER_CELL[args.precision]
    achieved = bpc * cells / (ms * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": round(cells / (ms * 1e-3) / 1e6, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32", "f16dev": "f32 (f16 storage)", "f64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "sediment_paper_d26_104x1040_3ratios_SI_and_ME", "cases": n, "cells": cells,
                   "rho_r": list(W.PAPER_SED_RATIOS), "tau": 0.6, "eta": 1e-6, "g_lattice": g,
                   "si_points": len(cases[0].si_ds), "force_source": ["SI", "ME"], "storage": args.precision,
                   "streaming": args.streaming.upper(),
                   "parallelism": "single GPU, one batched step and one batched body launch per step"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_step_batch",
                     "kernel_us": round(ms * 1e3, 3), "bytes_per_cell": bpc, "cells_per_launch": cells},
        "bodies": bodies,
    }
    batch.close()
    for lat in lats:
        lat.close()
    return out


def run_serve(args, W):
    """Continuous batching of a Poisson request mix under an HBM budget, and
    the same trace served one request at a time."""
    from paper_2110_00967_amd.serve import GpuEngine, Server, serial_run, summarize

    reqs = W.serving_trace(nreq=args.requests, seed=0, rate=args.rate, steps_range=(2e3, 2e4))
    items = W.serving_items(reqs)
    eng = GpuEngine(args.precision, streaming=1 if args.streaming == "aa" else 0)
    # warm the kernels up once (first launches pay code-object loading)
    warm = items[0][2]
    h = eng.create(warm)
    eng.step([h], [10])
    eng.sync()
    eng.release(h)
    budget = int(args.budget_gib * 2 ** 30)
    served = summarize(Server(eng, budget, chunk=args.chunk, policy=args.policy,
                              saturate_cells=args.saturate_cells).run(items))
    serial = summarize(serial_run(eng, items))
    return {
        "metric": METRIC, "value": round(served["aggregate_MLUPS"], 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": sum(r["steps"] for r in reqs), "warmup": 10, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32", "f16dev": "f32 (f16 storage)", "f64": "f64"}[args.precision], "data": "synthetic",
        "config": {"workload": "serving_poisson_mix", "requests": args.requests, "rate_per_s": args.rate,
                   "grids": [[256, 256], [512, 256], [1024, 512], [2048, 1024]], "steps_range": [2000, 20000],
                   "hbm_budget_GiB": args.budget_gib, "chunk_steps": args.chunk, "policy": args.policy,
                   "saturate_cells": args.saturate_cells if args.policy == "srpt" else None,
                   "storage": args.precision, "streaming": args.streaming.upper()},
        "serving": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in served.items()},
        "serial": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in serial.items()},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", default="f32", choices=["f32", "f16dev", "f64"])
    ap.add_argument("--tile", default=None, help="step workgroup BXxBY: threads (cells) along x times rows")
    ap.add_argument("--requests", type=int, default=200, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=10.0, help="serve: Poisson arrival rate (requests/s)")
    ap.add_argument("--budget-gib", type=float, default=4.0, help="serve: HBM budget for resident lattices")
    ap.add_argument("--policy", default="fair", choices=["fair", "srpt"],
                    help="serve: run all resident lattices each chunk, or least remaining work first")
    ap.add_argument("--saturate-cells", type=int, default=4 << 20,
                    help="serve, srpt: cells a chunk's lattices must hold before the policy stops adding")
    ap.add_argument("--chunk", type=int, default=1000, help="serve: steps per chunk")
    ap.add_argument("--streaming", default="ab", choices=["ab", "aa"],
                    help="population storage of single-lattice workloads: two buffers or one (AA pattern)")
    ap.add_argument("--sed-seconds", type=float, default=0.0,
                    help="sediment-paper: also run to this physical time and report each disk's Reynolds number")
    ap.add_argument("--workload", default="naca",
                    choices=["naca", "sediment", "roofline", "disk", "sweep", "paper", "sediment-paper", "serve"],
                    help="naca: NACA 0012 2000x1000 (default); sediment: free disk 400x2000; "
                         "roofline: NACA 0012 chord 819 on 8192x8192; disk: 128x64 disk channel; "
                         "sweep: 64 airfoils (chords 100/150/200, AoA 0-20 deg) in one batched launch; "
                         "paper: the paper's full-scale airfoil runs (chord 278, 3614x1946, TRT, AoA 0-28 deg, "
                         "15 cases) in one batched launch; "
                         "serve: Poisson mix of airfoil and sedimentation requests, continuous batching")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_2110_00967_amd import vplbm as V

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)

    if args.workload in ("sweep", "paper"):
        print(json.dumps(run_sweep(args, torch, W, V, paper=args.workload == "paper")), flush=True)
        return
    if args.workload == "sediment-paper":
        print(json.dumps(run_sed_paper(args, torch, W, V)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(run_serve(args, W)), flush=True)
        return
    if args.workload == "naca":
        case = W.case_naca(chord=200, aoa_deg=10.0)
    elif args.workload == "sediment":
        case = W.case_sedimentation()
    elif args.workload == "roofline":
        case = W.case_naca(chord=819, aoa_deg=10.0)
        case.nx = case.ny = 8192
    else:
        case = W.case_disk_channel()
    cells = case.nx * case.ny
    aa = args.streaming == "aa"
    lat = V.Lattice.from_case(case, precision=args.precision, streaming=V.STREAM_AA if aa else V.STREAM_AB)
    if args.tile:
        bx, by = (int(v) for v in args.tile.split("x"))
        lat.set_tile(bx, by)

    lat.step(args.warmup)
    lat.sync()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    lat.step(args.steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ms_per_step = ms / args.steps
    mlups = cells / (ms_per_step * 1e-3) / 1e6

    # A static body runs exactly one kernel per step (the fused step kernel;
    # its forces are summed by the next launch), so the events around the
    # timed region give that kernel's average duration per launch, launch
    # gaps included.  A second pass brackets every launch with its own pair
    # of events (reported for reference; the extra event packets add a few
    # microseconds per launch).
    kn = min(args.steps, 1000)
    k_pairs_us = lat.step_timed(kn) / kn * 1e3
    # a moving body adds its own kernels to every step: use the per-launch pairs
    k_us = ms_per_step * 1e3 if case.rho_s is None else k_pairs_us
    bpc = BYTES_PER_CELL[args.precision]
    achieved = bpc * cells / (k_us * 1e-6) / 1e9
    traffic_bytes = measured_traffic() if (args.workload, args.precision, aa) == ("naca", "f32", False) else None
    traffic = None if traffic_bytes is None else round(traffic_bytes / (k_us * 1e-6) / 1e9, 1)
    me, si = lat.forces_me(), lat.forces_si()
    q = 0.5 * case.u_ref ** 2 * case.length_scale
    finite = bool(np.isfinite(me).all() and np.isfinite(si).all())

    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "f16dev": "f32 (f16 storage)", "f64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"{case.name}_{case.nx}x{case.ny}", "nx": case.nx, "ny": case.ny,
                   "storage": args.precision, "si_points": len(case.si_ds), "tau": round(case.tau, 4),
                   "eta": case.eta, "streaming": "AA (one buffer)" if aa else "AB (two buffers)",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_bytes_per_launch": traffic_bytes, "algorithmic_bytes_per_launch": bpc * cells,
                     "kernel": "k_step", "kernel_us": round(k_us, 3), "kernel_us_event_pairs": round(k_pairs_us, 3),
                     "bytes_per_cell": bpc, "cells_per_launch": cells},
        "forces": {"CD_ME": me[0] / q, "CL_ME": me[1] / q, "CD_SI": si[0] / q, "CL_SI": si[1] / q,
                   "finite": finite, "steps_run": lat.step_count},
    }
    lat.close()
    if args.copy_calibration:
        # plain streaming kernels of known size (read n bytes, write n bytes):
        # reference for the HBM byte counters and a measured copy ceiling
        cal = {}
        for nbytes in (1 << 30, 73 << 20):
            src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
            dst = torch.empty_like(src)
            torch.add(src, 1.0, out=dst)
            torch.cuda.synchronize()
            c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            c0.record()
            for _ in range(10):
                torch.add(src, 1.0, out=dst)
            c1.record()
            torch.cuda.synchronize()
            cal[f"{nbytes >> 20}MiB"] = {"bytes_read": nbytes, "bytes_written": nbytes, "launches": 10,
                                         "GBps": round(2 * nbytes * 10 / (c0.elapsed_time(c1) * 1e-3) / 1e9, 1)}
            del src, dst
        out["copy_calibration"] = cal
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(case)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
