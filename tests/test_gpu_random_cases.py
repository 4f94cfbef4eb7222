"""Seeded random configurations against the oracle (FP64): edge kinds per
axis (periodic in pairs, else velocity / free-slip / zero-gradient /
convective, chosen per edge), wall and convection speeds, tau, TRT, eta
(including +inf), a disk with stress-integration points on either stencil
rule, two-buffer or AA storage, random initial fields.  Each case runs 7
(odd) then 12 (even) steps; bars as in test_gpu_parity (populations 1e-12,
forces 1e-10 of their scale, bit-exact solid and sample-node sets)."""
import math

import numpy as np
import pytest

import workloads as W
from gpu_cases import P, V_, F, OUT, CV, build_gpu, build_oracle, random_fields, say, spec
from test_gpu_parity import compare_fp64

pytestmark = pytest.mark.gpu

NCASES = 24


def random_spec(k):
    rng = np.random.default_rng(1000 + k)
    nx, ny = (int(v) for v in rng.integers(30, 90, 2))

    def pair():
        if rng.random() < 0.3:
            return (P, 0.0, 0.0), (P, 0.0, 0.0)
        out = []
        for _ in range(2):
            kind = int(rng.choice([V_, F, OUT, CV]))
            if kind == V_:
                out.append((V_, float(rng.uniform(-0.04, 0.04)), float(rng.uniform(-0.04, 0.04))))
            elif kind == CV:
                out.append((CV, float(rng.uniform(0.0, 0.1)), 0.0))
            else:
                out.append((kind, 0.0, 0.0))
        return tuple(out)

    (w, e), (s_, n) = pair(), pair()
    tau = float(rng.uniform(0.52, 1.2))
    trt = float(rng.choice([0.0, 3.0 / 16.0, 1.0 / 6.0]))
    eta = float(rng.choice([1e-4, 1e-2, math.inf]))
    r = float(rng.uniform(3.0, min(nx, ny) / 2.0 - 8.0))
    m = r + 7.0  # room for links, sample walks and the interpolation point
    xc, yc = float(rng.uniform(m, nx - m)), float(rng.uniform(m, ny - m))
    npts = int(rng.integers(8, 64))
    rule = int(rng.integers(0, 2))
    aa = int(rng.integers(0, 2))
    fields = random_fields(nx, ny, 20 + k, amp=0.02)
    return spec(nx, ny, tau=tau, eta=eta, edges=(w, e, s_, n), trt=trt, si_rule=rule, disk=(xc, yc, r),
                si=W.disk_si_points(xc, yc, r, npts), init=("fields",) + fields), aa


@pytest.mark.parametrize("k", range(NCASES))
def test_random_case_fp64_against_oracle(k):
    s, aa = random_spec(k)
    say(f"random case {k}: {s['nx']}x{s['ny']} edges {s['edges']} tau {s['tau']:.3f} trt {s['trt']:.4f} "
        f"eta {s['eta']} disk {s['disk']} rule {s['si_rule']} {'AA' if aa else 'AB'}")
    g = build_gpu(s, "f64", streaming=aa)
    o = build_oracle(s)
    assert np.array_equal(g.mask() & 1, o.solid)
    sample = np.zeros(o.nx * o.ny, bool)
    sample[o.si_node] = True
    assert np.array_equal((g.mask().ravel() & 0x40) != 0, sample)
    for n in (7, 5):
        g.step(n)
        o.step(n)
        compare_fp64(g, o, f"random case {k} after {g.step_count}")
    g.close()
