"""Writes shedding_re100.json: long-horizon statistics of the FP64 oracle on
the Re = 100 shedding cylinder (workloads.case_cylinder_shedding).

After shedding sets in, runs in different precisions drift apart point by
point but keep the same statistics; the GPU test compares its own run with
these numbers.  Calls only the oracle (inputs from workloads).

    python tests/golden/make_shedding_golden.py     # about 6 minutes on 8 cores
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

WINDOW = (14000, 38000)  # steps: shedding established, about 10 periods


def coefficients(hist, case):
    """(C_D, C_L) time series from a force history (steps x 3)."""
    q = 0.5 * case.u_ref ** 2 * case.length_scale
    return hist[:, 0] / q, hist[:, 1] / q


def shedding_stats(cd, cl, case, window=WINDOW):
    """Mean C_D, mean C_L, C_L RMS about its mean, and the Strouhal number
    D / (U T) with T the mean spacing of upward crossings of C_L through its
    mean (linear interpolation between steps) inside the window."""
    a, b = window
    cd, cl = cd[a:b], cl[a:b]
    m = cl.mean()
    s = cl - m
    up = np.nonzero((s[:-1] < 0) & (s[1:] >= 0))[0]
    t = up + (-s[up]) / (s[up + 1] - s[up])
    period = (t[-1] - t[0]) / (len(t) - 1)
    return {"cd_mean": float(cd.mean()), "cl_mean": float(m), "cl_rms": float(np.sqrt((s * s).mean())),
            "strouhal": float(case.length_scale / (case.u_ref * period)), "periods": int(len(t) - 1)}


def main():
    import oracle as O
    import workloads as W

    case = W.case_cylinder_shedding()
    o = O.RefLattice.from_case(case)
    o.set_fields(*W.shedding_initial_fields(case))
    while o.nstep < case.steps:
        o.step(2000)
        print(o.nstep, flush=True)
    out = {"case": case.name, "steps": case.steps, "window": list(WINDOW), "source": "FP64 oracle"}
    for name, hist in (("si", o.si()), ("me", o.me())):
        out[name] = shedding_stats(*coefficients(hist, case), case)
    with open(os.path.join(HERE, "shedding_re100.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
