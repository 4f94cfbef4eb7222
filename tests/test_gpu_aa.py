"""AA-pattern storage (one population buffer updated in place).

Each step does the same arithmetic on the same values as the two-buffer
path; only the compiler's fusion of multiplies and adds may differ between
the kernels, so results agree to rounding, not bit for bit.  Bars:
  * against the oracle, every two-buffer parity case in FP64 at its bars
    (populations 1e-12, forces 1e-10 of their scale), checked after odd step
    counts (state pushed to the neighbours) and even ones (state swapped in
    the cell);
  * against the two-buffer path in FP32 / FP16 storage, derived from the
    storage rounding (a few ulps of a population, propagated over the run).
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from gpu_cases import build_gpu, build_oracle, oracle_pops, rel_l2, say
from test_gpu_parity import FP64_FORCE, FP64_POP, RAGGED, compare_fp64

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", sorted(RAGGED))
def test_aa_fp64_against_oracle(name):
    s = RAGGED[name]
    say("AA fp64 vs oracle", name, f"{s['nx']}x{s['ny']}")
    g = build_gpu(s, "f64", streaming=1)
    o = build_oracle(s)
    compare_fp64(g, o, f"{name} AA initial")
    for n in (1, 6, 7, 19):  # after 1, 7 (odd), 14 (even) and 33 (odd) steps
        g.step(n)
        o.step(n)
        compare_fp64(g, o, f"{name} AA after {g.step_count}")
    if s["si"] is not None:
        # one-shot stress integration from the odd-step layout (33 steps) and
        # the even one (34): each equals the SI the next step computes
        xy, nrm, ds = s["si"]
        for _ in range(2):
            ref = g.forces_si_at(xy, nrm, ds)
            g.step(1)
            assert np.abs(ref - g.forces_si()).max() <= 1e-12 * max(np.abs(ref).max(), 1e-3)
    g.close()


@pytest.mark.parametrize("precision,pop_bar,force_bar", [("f32", 1e-6, 1e-5), ("f16dev", 5e-4, 1e-2)])
@pytest.mark.parametrize("name", ["inlet_outlet_freeslip_naca", "convective_trt_naca", "couette_walls_force",
                                  "convective_east_and_north_corner"])
def test_aa_against_two_buffer_reduced_precision(name, precision, pop_bar, force_bar):
    s = RAGGED[name]
    say("AA vs AB", precision, name)
    ab, aa = build_gpu(s, precision), build_gpu(s, precision, streaming=1)
    assert np.array_equal(ab.populations(), aa.populations())  # same initial state, either layout
    for n in (13, 40):
        ab.step(n, macro=True)
        aa.step(n, macro=True)
        e = np.abs(ab.populations() - aa.populations()).max()
        assert e <= pop_bar, (name, precision, ab.step_count, e)
        for w in (0, 1):
            ha, hb = ab.history(w), aa.history(w)
            scale = max(np.abs(ha).max(), 1e-3)
            assert np.abs(ha - hb).max() <= force_bar * scale, (name, precision, w)
        (ra, ua, va), (rb, ub, vb) = ab.macro(), aa.macro()
        assert rel_l2(np.stack([ub, vb]), np.stack([ua, va])) <= 100 * pop_bar
    ab.close()
    aa.close()


@pytest.mark.parametrize("source", [0, 1])
def test_aa_free_disk_fp64_against_oracle(source):
    from gpu_cases import O
    from paper_2110_00967_amd import vplbm as V
    case = W.case_sedimentation(nx=80, ny=200, d=12.0, g=2e-4, y0=150.0, steps=300, npts=48,
                                force_source=source)
    say("AA free disk fp64 vs oracle, source", source)
    o = O.RefLattice.from_case(case)
    g = V.Lattice.from_case(case, precision="f64", streaming=V.STREAM_AA)
    for n in (101, 100):  # odd, then even
        g.step(n)
        o.step(n)
        bg, bo = g.body_state(), o.body_state()
        assert np.abs(bg - bo).max() <= 1e-10 * max(1.0, np.abs(bo).max()), (bg, bo)
        assert np.array_equal(g.mask() & 1, o.solid)
        compare_fp64(g, o, f"AA free disk after {g.step_count}")
    g.close()


def test_aa_paper_scale_sedimentation_fp32():
    from paper_2110_00967_amd import vplbm as V
    case = W.case_sedimentation_paper(rho_r=1.03)
    say("AA vs AB paper-scale sedimentation fp32, 301 steps")
    ab = V.Lattice.from_case(case, precision="f32")
    aa = V.Lattice.from_case(case, precision="f32", streaming=V.STREAM_AA)
    ab.step(301)
    aa.step(301)
    ba, bb = ab.body_state(), aa.body_state()
    assert abs(ba[4] - bb[4]) <= 1e-5 * abs(ba[4])
    assert np.abs(ab.populations() - aa.populations()).max() <= 1e-6
    ab.close()
    aa.close()


def test_aa_rejections():
    from paper_2110_00967_amd import vplbm as V
    say("AA rejections")
    p = V.make_params(64, 32, 0.7, 1e-4, precision="f32", streaming=V.STREAM_AA)
    g = V.Lattice(p)
    with pytest.raises(V.VplbmError) as e:
        g.set_tile(128, 2)
    assert e.value.code == V.EINVAL
    g.set_tile(64, 4)
    g.init_uniform(1.0, 0.01, 0.0)
    g.step(3)
    assert np.isfinite(g.populations()).all()
    g.close()
