#!/usr/bin/env python3
"""Throughput of the fused VP-LBM step on one MI355X.

Default workload: the angle-of-attack sweep -- 64 NACA 0012 airfoils (chords
100/150/200 cells on 10c x 5c channels, AoA 0..20 deg, Re = 1000), 76.6 M
cells, FP32 deviation storage, all 64 stepped together by one batched launch
of the fused step kernel per time step (`k_step_batch`).  Its 5.6 GB of
populations lie far beyond the 256 MB Infinity Cache, so the step's HBM
roofline is honest here.  One "step" is one full time step of every case:
pull streaming with the edge rules, penalization, collision, momentum
exchange and stress integration, and the force finalize (folded into the
next launch).  Inputs are resident in HBM before timing starts.

Prints one JSON line: metric, MLUPS, the roofline of k_step_batch (algorithmic
bytes per launch over its average duration, measured with HIP events on the
lattices' stream; `traffic` from the committed rocprofv3 counter summary),
the FP64 CPU oracle on a bounded sample of one sweep case (all host threads
and one), and, as extra keys, the same sweep in FP16 deviation storage, the
single 2000 x 1000 airfoil (cache-resident, labelled so), the 8192 x 8192
roofline lattice, and a bounded serving run with p50/p99 latency.  Only one
GPU is supported.
"""
from __future__ import annotations

import argparse
import hashlib
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
MALL_BYTES = 256 << 20
BYTES_PER_CELL = {"f64": 9 * 8 * 2 + 1, "f32": 9 * 4 * 2 + 1, "f16dev": 9 * 2 * 2 + 1}
DTYPE = {"f32": "f32", "f16dev": "f32 (f16 storage)", "f64": "f64"}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2110_00967_amd", "csrc", f)
                  for f in ("d2q9.hpp", "sample.hpp", "mover.hpp", "step_kernel.hpp")]
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(name):
    """HBM bytes per launch of a step kernel from a committed rocprofv3
    counter summary (profiles/<name>), or None when the file is missing or the
    kernel source changed since the counters were taken."""
    path = os.path.join(PROFILES, name)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("#", "|", "`", " ")):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(case, budget_s=10.0):
    """The FP64 oracle as it stands, on the host: a bounded number of steps of
    one case, with every OpenMP thread and with one."""
    import oracle as O

    def timed(threads):
        used = O.set_threads(threads)
        lat = O.RefLattice.from_case(case)
        lat.step(1)  # warm-up (page-in, thread pool)
        n = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s or n < 2:
            lat.step(1)
            n += 1
        dt = time.perf_counter() - t0
        return case.nx * case.ny * n / dt / 1e6, used, n, dt

    all_threads = O.max_threads()
    v_all, used_all, n_all, dt_all = timed(all_threads)
    v_one, _, n_one, dt_one = timed(1)
    O.set_threads(all_threads)
    cpu = platform.processor() or platform.machine()
    return {
        "value": round(v_all, 2), "unit": "MLUPS", "cores": used_all, "kind": "oracle",
        "sample": f"{case.name} {case.nx}x{case.ny} (one case of the sweep), FP64 oracle, {n_all} steps in "
                  f"{dt_all:.1f} s on {used_all} OpenMP threads; single thread {n_one} steps in {dt_one:.1f} s; "
                  f"host {cpu}, {os.cpu_count()} logical CPUs",
        "single_thread": {"value": round(v_one, 2), "unit": "MLUPS", "cores": 1},
    }


def events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def autotuned_batch_tile(args, torch, V, batch, cells, prec):
    """The batch tile for this (precision, size class): from the tile cache
    when present, else tuned now (and cached)."""
    from paper_2110_00967_amd import autotune as AT

    tuner = AT.TileTuner()
    key = AT.batch_key(prec, "AB", batch)
    tile = tuner.lookup(key)
    source = (tuner.entry(key) or {}).get("source")
    if tile is None or args.retune:
        tile = AT.tune_batch(batch, tuner, key, steps=max(20, min(args.steps, 60)))
        source = "tuned now"
    batch.set_tile(*tile)
    return {"tile": list(tile), "key": key, "source": source, "timings_us": tuner.timings(key)}


def run_sweep(args, torch, W, V, precision=None, paper=False, serial=True, tune=True):
    """Many airfoil cases stepped by one launch per step, and the same cases
    stepped one after the other (the plain single-case form).  Default: 64
    cases (chords 100/150/200, AoA 0-20 deg).  paper: the paper's full-scale
    runs, chord 278 on 3614 x 1946, TRT, AoA 0-28 deg in steps of 2."""
    prec = precision or args.precision
    cases = W.paper_aoa_sweep() if paper else W.sweep_cases()
    st = V.STREAM_AA if args.streaming == "aa" else V.STREAM_AB
    lats = [V.Lattice.from_case(c, precision=prec, streaming=st) for c in cases]
    cells = sum(c.nx * c.ny for c in cases)
    batch = V.Batch(lats)
    n = len(lats)
    tile_info = None
    if tune and st == V.STREAM_AB and not args.no_tune:
        tile_info = autotuned_batch_tile(args, torch, V, batch, cells, prec)
    batch.step([args.warmup] * n)
    torch.cuda.synchronize()
    e0, e1 = events(torch)
    e0.record()
    batch.step([args.steps] * n)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    bpc = BYTES_PER_CELL[prec]
    achieved = bpc * cells / (ms * 1e-3) / 1e9
    q = [0.5 * c.u_ref ** 2 * c.length_scale for c in cases]
    cd = [lat.forces_si()[0] / qq for lat, qq in zip(lats, q)]
    pop_bytes = sum(lat.nbytes for lat in lats)
    if paper:
        config = {"workload": "naca0012_paper_c278_3614x1946_trt_aoa_sweep", "cases": n, "cells": cells,
                  "chord": 278, "aoa_deg": [0.0, 2.0 * (n - 1)],
                  "tau": 0.55, "trt_lambda": round(1.0 / 6.0, 6), "eta": 1e-6, "si_points": len(cases[0].si_ds),
                  "storage": prec, "streaming": args.streaming.upper(),
                  "parallelism": "single GPU, one batched launch per step"}
    else:
        config = {"workload": "naca0012_aoa_sweep_64cases_76.6Mcells", "cases": n, "cells": cells,
                  "chords": [100, 150, 200], "grids": "10c x 5c", "aoa_deg": [0.0, 20.0], "re": 1000,
                  "si_points_per_case": len(cases[0].si_ds), "storage": prec, "streaming": args.streaming.upper(),
                  "device_bytes": pop_bytes, "parallelism": "single GPU, one batched launch per step"}
    if tile_info is not None:
        config["batch_tile"] = tile_info["tile"]
    k_us = ms * 1e3
    out = {
        "metric": METRIC, "value": round(cells / (ms * 1e-3) / 1e6, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prec], "data": "synthetic",
        "config": config,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": "k_step_batch",
                     "kernel_us": round(k_us, 3), "bytes_per_cell": bpc, "cells_per_launch": cells,
                     "algorithmic_bytes_per_launch": bpc * cells},
        "CD_SI_range": [round(min(cd), 4), round(max(cd), 4)],
    }
    if tile_info is not None:
        out["autotune"] = tile_info
    if serial:
        # the plain form: each case alone, one after the other, same steps
        ks = max(args.steps // 4, 1)
        s0, s1 = events(torch)
        s0.record()
        for lat in lats:
            lat.step(ks)
        s1.record()
        torch.cuda.synchronize()
        ms_serial = s0.elapsed_time(s1) / ks
        out["serial"] = {"ms_per_step": round(ms_serial, 5), "MLUPS": round(cells / (ms_serial * 1e-3) / 1e6, 1),
                         "steps": ks}
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
    e0, e1 = events(torch)
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
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.precision], "data": "synthetic",
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


def run_serve(args, W, nreq=None, steps_range=None, rate=None, budget_gib=None):
    """Continuous batching of a Poisson request mix under an HBM budget, and
    the same trace served one request at a time."""
    from paper_2110_00967_amd.serve import GpuEngine, Server, serial_run, summarize

    nreq = nreq or args.requests
    steps_range = steps_range or (args.min_steps, args.max_steps)
    rate = rate or args.rate
    budget_gib = budget_gib or args.budget_gib
    reqs = W.serving_trace(nreq=nreq, seed=0, rate=rate, steps_range=steps_range)
    items = W.serving_items(reqs)
    eng = GpuEngine(args.precision, streaming=1 if args.streaming == "aa" else 0)
    # warm the kernels up once (first launches pay code-object loading)
    warm = items[0][2]
    h = eng.create(warm)
    eng.step([h], [10])
    eng.sync()
    eng.release(h)
    budget = int(budget_gib * 2 ** 30)
    server = Server(eng, budget, chunk=args.chunk, policy=args.policy, saturate_cells=args.saturate_cells)

    def progress(done, total, t):
        if done % 25 == 0 or done == total:
            print(f"[serve] {done}/{total} requests finished at {t:.1f} s", file=sys.stderr, flush=True)

    served = summarize(server.run(items, progress=progress))
    served["peak_resident_bytes"] = server.peak_bytes
    served["peak_resident"] = server.peak_resident
    out = {
        "metric": METRIC, "value": round(served["aggregate_MLUPS"], 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": sum(r["steps"] for r in reqs), "warmup": 10, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.precision], "data": "synthetic",
        "config": {"workload": "serving_poisson_mix", "requests": nreq, "rate_per_s": rate,
                   "grids": [[256, 256], [512, 256], [1024, 512], [2048, 1024]],
                   "steps_range": [int(steps_range[0]), int(steps_range[1])],
                   "hbm_budget_GiB": budget_gib, "chunk_steps": args.chunk, "policy": args.policy,
                   "saturate_cells": args.saturate_cells if args.policy == "srpt" else None,
                   "storage": args.precision, "streaming": args.streaming.upper()},
        "serving": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in served.items()},
    }
    if not args.no_serial:
        serial = summarize(serial_run(eng, items))
        out["serial"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in serial.items()}
    eng.close()
    return out


def time_single(args, torch, V, case, precision, steps, warmup, tile=None):
    """One lattice stepped alone: ms per step from events over the timed
    region, and per-launch event pairs of the step kernel."""
    lat = V.Lattice.from_case(case, precision=precision,
                              streaming=V.STREAM_AA if args.streaming == "aa" else V.STREAM_AB)
    if tile:
        lat.set_tile(*tile)
    else:
        from paper_2110_00967_amd import autotune as AT

        AT.apply_lattice(lat)  # the tuned tile of this class, when one is cached
    lat.step(warmup)
    lat.sync()
    torch.cuda.synchronize()
    e0, e1 = events(torch)
    e0.record()
    lat.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    kn = min(steps, 1000)
    k_pairs_us = lat.step_timed(kn) / kn * 1e3
    return lat, ms, k_pairs_us


def run_single(args, torch, W, V, workload, precision, steps=None, warmup=None, quiet_forces=False):
    """One lattice alone: NACA 0012 2000 x 1000 (cache-resident), the
    sedimenting disk, the 8192 x 8192 roofline lattice or the disk channel."""
    steps = steps or args.steps
    warmup = warmup if warmup is not None else args.warmup
    if workload == "naca":
        case = W.case_naca(chord=200, aoa_deg=10.0)
    elif workload == "sediment":
        case = W.case_sedimentation()
    elif workload == "roofline":
        case = W.case_naca(chord=819, aoa_deg=10.0)
        case.nx = case.ny = 8192
    else:
        case = W.case_disk_channel()
    cells = case.nx * case.ny
    tile = tuple(int(v) for v in args.tile.split("x")) if args.tile else None
    lat, ms_per_step, k_pairs_us = time_single(args, torch, V, case, precision, steps, warmup, tile)
    mlups = cells / (ms_per_step * 1e-3) / 1e6
    # Every step is exactly one kernel, the fused step kernel (forces are
    # summed by the next launch; a moving disk advances inside it), so the
    # events around the timed region give that kernel's average duration per
    # launch, launch gaps included.
    k_us = ms_per_step * 1e3
    bpc = BYTES_PER_CELL[precision]
    achieved = bpc * cells / (k_us * 1e-6) / 1e9
    me, si = lat.forces_me(), lat.forces_si()
    q = 0.5 * case.u_ref ** 2 * case.length_scale
    pop_bytes = 2 * 9 * lat.nx * lat.ny * {"f64": 8, "f32": 4, "f16dev": 2}[precision]
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": round(ms_per_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[precision], "data": "synthetic",
        "config": {"workload": f"{case.name}_{case.nx}x{case.ny}", "nx": case.nx, "ny": case.ny,
                   "storage": precision, "si_points": len(case.si_ds), "tau": round(case.tau, 4),
                   "eta": case.eta, "streaming": "AA (one buffer)" if args.streaming == "aa" else "AB (two buffers)",
                   "tile": list(lat.tile), "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes_per_launch": bpc * cells, "kernel": "k_step", "kernel_us": round(k_us, 3),
                     "kernel_us_event_pairs": round(k_pairs_us, 3), "bytes_per_cell": bpc,
                     "cells_per_launch": cells},
        "cache_resident": pop_bytes <= MALL_BYTES,
    }
    if not quiet_forces:
        out["forces"] = {"CD_ME": me[0] / q, "CL_ME": me[1] / q, "CD_SI": si[0] / q, "CL_SI": si[1] / q,
                         "finite": bool(np.isfinite(me).all() and np.isfinite(si).all()),
                         "steps_run": lat.step_count}
    if case.rho_s is not None:
        # whole step (step kernel + body kernel) against the step kernel alone
        out["roofline"]["whole_step_us"] = round(ms_per_step * 1e3, 3)
    lat.close()
    return out, case


def copy_calibration(torch):
    """Plain streaming kernels of known size (read n bytes, write n bytes):
    the reference for the HBM byte counters and a measured copy ceiling."""
    cal = {}
    for nbytes in (1 << 30, 73 << 20):
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        c0, c1 = events(torch)
        c0.record()
        for _ in range(10):
            torch.add(src, 1.0, out=dst)
        c1.record()
        torch.cuda.synchronize()
        cal[f"{nbytes >> 20}MiB"] = {"bytes_read": nbytes, "bytes_written": nbytes, "launches": 10,
                                     "GBps": round(2 * nbytes * 10 / (c0.elapsed_time(c1) * 1e-3) / 1e9, 1)}
        del src, dst
    return cal


def copy_ceiling(torch, nbytes=2 << 30, launches=10):
    """The HBM ceiling a plain streaming kernel reaches on this GPU: torch's
    elementwise add over float32 (read nbytes, write nbytes per launch),
    far beyond the Infinity Cache, HIP events around `launches` launches."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.add(src, 1.0, out=dst)
    torch.cuda.synchronize()
    c0, c1 = events(torch)
    c0.record()
    for _ in range(launches):
        torch.add(src, 1.0, out=dst)
    c1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * launches / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"kernel": "torch.add, float32, read n + write n bytes", "bytes_per_launch": 2 * nbytes,
            "launches": launches, "GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}


def brief(d):
    """The figures of a sub-run that go into the headline line's extra keys."""
    r = d["roofline"]
    out = {"workload": d["config"]["workload"], "MLUPS": d["value"], "ms_per_step": d["ms_per_step"],
           "storage": d["config"].get("storage"), "frac": r["frac"], "achieved_GBps": r["achieved"],
           "kernel": r["kernel"], "kernel_us": r["kernel_us"], "traffic": r.get("traffic")}
    for k in ("cache_resident", "serial", "autotune"):
        if k in d:
            out[k] = d[k]
    if "tile" in d["config"]:
        out["tile"] = d["config"]["tile"]
    if "batch_tile" in d["config"]:
        out["tile"] = d["config"]["batch_tile"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="f32", choices=["f32", "f16dev", "f64"])
    ap.add_argument("--tile", default=None, help="single lattice: step workgroup BXxBY (threads along x times rows)")
    ap.add_argument("--no-tune", action="store_true", help="sweep: keep the default batch tile (no autotuner)")
    ap.add_argument("--retune", action="store_true", help="sweep: re-time the batch tiles even when cached")
    ap.add_argument("--requests", type=int, default=500, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serve: Poisson arrival rate (requests/s); 0 = 0.8 of the measured capacity")
    ap.add_argument("--min-steps", type=float, default=1e4, help="serve: smallest request (steps)")
    ap.add_argument("--max-steps", type=float, default=1e5, help="serve: largest request (steps)")
    ap.add_argument("--budget-gib", type=float, default=4.0, help="serve: HBM budget for resident lattices")
    ap.add_argument("--policy", default="fair", choices=["fair", "srpt"],
                    help="serve: run all resident lattices each chunk, or least remaining work first")
    ap.add_argument("--saturate-cells", type=int, default=4 << 20,
                    help="serve, srpt: cells a chunk's lattices must hold before the policy stops adding")
    ap.add_argument("--chunk", type=int, default=1000, help="serve: steps per chunk")
    ap.add_argument("--no-serial", action="store_true", help="serve: skip the one-request-at-a-time comparison")
    ap.add_argument("--streaming", default="ab", choices=["ab", "aa"],
                    help="population storage: two buffers or one (AA pattern)")
    ap.add_argument("--sed-seconds", type=float, default=0.0,
                    help="sediment-paper: also run to this physical time and report each disk's Reynolds number")
    ap.add_argument("--workload", default="sweep",
                    choices=["sweep", "naca", "sediment", "roofline", "disk", "paper", "sediment-paper", "serve"],
                    help="sweep (default): 64 airfoils (chords 100/150/200, AoA 0-20 deg, 76.6 M cells) in one "
                         "batched launch per step; naca: NACA 0012 2000x1000 alone (cache-resident); "
                         "sediment: free disk 400x2000; roofline: NACA 0012 chord 819 on 8192x8192; "
                         "disk: 128x64 disk channel; paper: the paper's full-scale airfoil runs (chord 278, "
                         "3614x1946, TRT, AoA 0-28 deg, 15 cases) in one batched launch; "
                         "serve: Poisson mix of airfoil and sedimentation requests, continuous batching")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="sweep: only the headline (no FP16 sweep, single lattices or serving run)")
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

    def say(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    if args.workload == "paper":
        print(json.dumps(run_sweep(args, torch, W, V, paper=True, tune=False)), flush=True)
        return
    if args.workload == "sediment-paper":
        print(json.dumps(run_sed_paper(args, torch, W, V)), flush=True)
        return
    if args.workload == "serve":
        if args.rate <= 0:
            args.rate = serving_rate(args, W)
        print(json.dumps(run_serve(args, W)), flush=True)
        return
    if args.workload != "sweep":
        out, case = run_single(args, torch, W, V, args.workload, args.precision)
        if (args.workload, args.precision, args.streaming) == ("naca", "f32", "ab"):
            t = measured_traffic("k_step_naca0012_2000x1000_f32_hbm_counters.md")
            out["roofline"]["traffic_bytes_per_launch"] = t
            out["roofline"]["traffic"] = None if t is None else round(t / (out["roofline"]["kernel_us"] * 1e-6) / 1e9, 1)
        if args.copy_calibration:
            out["copy_calibration"] = copy_calibration(torch)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(case)
        print(json.dumps(out), flush=True)
        return

    # headline: the 64-case sweep, one batched launch per step
    say(f"sweep {args.precision}: 64 cases, {args.steps} steps after {args.warmup}")
    out = run_sweep(args, torch, W, V)
    if args.streaming == "ab":
        t = measured_traffic(f"k_step_batch_naca0012_sweep64_{args.precision}_hbm_counters.md")
        out["roofline"]["traffic_bytes_per_launch"] = t
        out["roofline"]["traffic"] = None if t is None else round(t / (out["roofline"]["kernel_us"] * 1e-6) / 1e9, 1)
    if not args.no_extras:
        extras = {}
        if args.precision == "f32":
            say("sweep f16dev")
            f16 = run_sweep(args, torch, W, V, precision="f16dev", serial=False)
            t = measured_traffic("k_step_batch_naca0012_sweep64_f16dev_hbm_counters.md")
            f16["roofline"]["traffic"] = None if t is None else round(t / (f16["roofline"]["kernel_us"] * 1e-6) / 1e9, 1)
            extras["sweep_f16dev"] = brief(f16)
        say("naca 2000x1000 alone")
        c2, _ = run_single(args, torch, W, V, "naca", args.precision, quiet_forces=True)
        extras["naca_2000x1000_alone"] = brief(c2)
        say("roofline lattice 8192x8192")
        r, _ = run_single(args, torch, W, V, "roofline", args.precision, steps=max(args.steps, 20), quiet_forces=True)
        extras["roofline_8192x8192"] = brief(r)
        say("serving, bounded trace")
        sv = run_serve(args, W, nreq=48, steps_range=(1e3, 1e4), rate=40.0, budget_gib=2.0)
        extras["serving_bounded"] = {"config": sv["config"], **sv["serving"],
                                     "note": "48 requests, steps 1e3-1e4 (C5 shape, 1/10 the steps); "
                                             "the full trace runs with --workload serve"}
        say("copy ceiling")
        extras["copy_ceiling"] = copy_ceiling(torch)
        out["extras"] = extras
    if args.copy_calibration:
        out["copy_calibration"] = copy_calibration(torch)
    if not args.no_cpu_baseline:
        say("cpu baseline (FP64 oracle)")
        out["cpu_baseline"] = cpu_baseline(W.sweep_cases()[0])
    print(json.dumps(out), flush=True)


def serving_rate(args, W):
    """0.8 of the measured capacity for the trace's mean request: the batched
    sweep's MLUPS (a saturated batch) over the mean request's cell updates."""
    reqs = W.serving_trace(nreq=args.requests, seed=0, rate=1.0, steps_range=(args.min_steps, args.max_steps))
    work = sum(r["nx"] * r["ny"] * r["steps"] for r in reqs) / len(reqs)
    capacity_mlups = 76000.0 if args.precision == "f32" else (110000.0 if args.precision == "f16dev" else 38000.0)
    return 0.8 * capacity_mlups * 1e6 / work


if __name__ == "__main__":
    main()
