"""Shared builders for the GPU-vs-oracle parity tests: one declarative case
description drives both the HIP library (through the C ABI binding) and the
CPU oracle, with the same seeded inputs."""
from __future__ import annotations

import math
import sys

import numpy as np

import oracle as O
import workloads as W

P, V_, F, OUT, CV = W.PERIODIC, W.VELOCITY, W.FREESLIP, W.OUTFLOW, W.CONVECTIVE


def say(*a):
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


def spec(nx, ny, tau=0.7, eta=1e-4, edges=((P, 0, 0),) * 4, **kw):
    d = dict(nx=nx, ny=ny, tau=tau, eta=eta, edges=edges, rho0=1.0, gx=0.0, gy=0.0, trt=0.0, si_rule=0, disk=None,
             polygon=None, ref=None, mask=None, si=None, motion=None, dynamics=None, init=("uniform", 1.0, 0.0, 0.0))
    d.update(kw)
    return d


def random_fields(nx, ny, seed, amp=0.03):
    ux, uy = W.smooth_random_velocity(nx, ny, seed=seed, amp=amp)
    rho = W.random_density(nx, ny, seed=seed + 1, amp=1e-3)
    return rho, ux, uy


def build_oracle(s):
    e = s["edges"]
    lat = O.RefLattice(s["nx"], s["ny"], s["tau"], s["eta"], s["rho0"], e[0], e[1], e[2], e[3], s["gx"], s["gy"],
                       s["trt"], s["si_rule"])
    _setup(lat, s, oracle=True)
    return lat


def build_gpu(s, precision="f64", **kw):
    from paper_2110_00967_amd import vplbm as V
    e = s["edges"]
    npts = 0 if s["si"] is None else len(s["si"][2])
    p = V.make_params(s["nx"], s["ny"], s["tau"], s["eta"], s["rho0"], precision, e[0], e[1], e[2], e[3],
                      max_si_points=max(16, npts), trt_lambda=s["trt"], si_rule=s["si_rule"], **kw)
    lat = V.Lattice(p)
    if s["gx"] or s["gy"]:
        lat.set_body_force(s["gx"], s["gy"])
    _setup(lat, s, oracle=False)
    return lat


def _setup(lat, s, oracle):
    if s["disk"] is not None:
        lat.set_disk(*s["disk"])
    elif s["polygon"] is not None:
        lat.set_polygon(s["polygon"], s["ref"])
    elif s["mask"] is not None:
        lat.set_mask(s["mask"])
    if s["si"] is not None:
        lat.set_si_points(*s["si"])
    if s["motion"] is not None:
        lat.set_motion(*s["motion"])
    if s["dynamics"] is not None:
        lat.set_dynamics(*s["dynamics"])
    kind = s["init"][0]
    if kind == "uniform":
        lat.init_uniform(*s["init"][1:])
    else:
        lat.set_fields(*s["init"][1:])


def oracle_pops(lat):
    return np.transpose(lat.ft, (2, 0, 1))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def small_naca(nx=150, ny=75, chord=30.0, aoa=10.0):
    poly = W.naca0012_polygon(chord, 0.3 * nx, 0.5 * ny, aoa, n_side=40)
    xy, n, ds = W.polygon_si_points(poly)
    cx, cy, _ = W.polygon_centroid(poly)
    return poly, (cx, cy), (xy, n, ds)
