"""Long-horizon statistics of the Re = 100 shedding cylinder against the FP64
oracle's, stored in tests/golden/shedding_re100.json (written by
tests/golden/make_shedding_golden.py, which runs only the oracle).

Once the wake sheds, runs in different precisions or rounding orders drift
apart point by point but keep the same statistics.  Bars, over about ten
shedding periods (steps 14,000-38,000): mean C_D and the Strouhal number
within 0.5%, mean C_L within 0.5% of C_D, C_L RMS within 2%; for both force
methods."""
import json
import os
import sys

import numpy as np
import pytest

import workloads as W
from gpu_cases import say

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from make_shedding_golden import coefficients, shedding_stats  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_shedding_statistics_match_oracle(precision):
    from paper_2110_00967_amd import vplbm as V
    with open(os.path.join(HERE, "golden", "shedding_re100.json")) as fh:
        ref = json.load(fh)
    case = W.case_cylinder_shedding()
    say("shedding cylinder Re 100", f"{case.nx}x{case.ny}", precision, case.steps, "steps")
    g = V.Lattice.from_case(case, precision=precision, hist_capacity=case.steps)
    g.set_fields(*W.shedding_initial_fields(case))
    g.step(case.steps)
    for name, which in (("si", V.FORCE_SI), ("me", V.FORCE_ME)):
        st = shedding_stats(*coefficients(g.history(which), case), case)
        r = ref[name]
        say(name, "gpu", st, "oracle", r)
        assert st["periods"] >= 8
        assert abs(st["cd_mean"] - r["cd_mean"]) <= 5e-3 * abs(r["cd_mean"])
        assert abs(st["strouhal"] - r["strouhal"]) <= 5e-3 * r["strouhal"]
        assert abs(st["cl_mean"] - r["cl_mean"]) <= 5e-3 * abs(r["cd_mean"])
        assert abs(st["cl_rms"] - r["cl_rms"]) <= 2e-2 * r["cl_rms"]
    g.close()
