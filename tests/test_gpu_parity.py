"""GPU-vs-oracle parity of the fused VP-LBM step, called through the C ABI.

Bars (FP64 storage and arithmetic, the oracle in FP64 with no FMA
contraction): populations within 1e-12 absolute, rho/u relative L2 within
1e-12, both force histories within 1e-10 of the largest force.  Integer and
byte work (solid indicator, sample nodes) must match bit for bit.
"""
import math

import numpy as np
import pytest

import workloads as W
from gpu_cases import (CV, F, OUT, P, V_, build_gpu, build_oracle, oracle_pops, random_fields, rel_l2, say,
                       small_naca, spec)

pytestmark = pytest.mark.gpu

FP64_POP = 1e-12
FP64_FIELD = 1e-12
FP64_FORCE = 1e-10


def compare_fp64(g, o, label, forces=True):
    fg = g.populations()
    fo = oracle_pops(o)
    err = np.abs(fg - fo).max()
    assert err <= FP64_POP, f"{label}: populations max err {err:.3e}"
    if forces and g.step_count:
        for which, ref in ((0, o.me()), (1, o.si())):
            h = g.history(which)
            # forces of real cases are >= 1e-3; cases at rest compare absolutely
            scale = max(np.abs(ref).max(), 1e-3)
            e = np.abs(h - ref[-len(h):]).max() / scale
            assert e <= FP64_FORCE, f"{label}: force {which} err {e:.3e} (scale {scale:.3e})"


def test_c1_disk_channel_fp64_full_length():
    case = W.case_disk_channel()
    say("disk channel 128x64 fp64", case.steps, "steps")
    o = W  # keep names short below
    from gpu_cases import O
    orc = O.RefLattice.from_case(case)
    from paper_2110_00967_amd import vplbm as V
    g = V.Lattice.from_case(case, precision="f64")
    assert (g.mask() & 1).sum() == 197
    for chunk in range(4):
        n = case.steps // 4
        g.step(n, macro=True)
        orc.step(n)
        r, u, v = g.macro()
        assert rel_l2(r, orc.rho) <= FP64_FIELD
        assert rel_l2(np.stack([u, v]), np.stack([orc.ux, orc.uy])) <= FP64_FIELD
    compare_fp64(g, orc, "disk channel")
    me, si = g.forces_me(), g.forces_si()
    q = 0.5 * case.u_ref ** 2 * case.length_scale
    say(f"C_D(ME)={me[0]/q:.6f} C_D(SI)={si[0]/q:.6f} C_L(ME)={me[1]/q:.2e} C_L(SI)={si[1]/q:.2e}")


RAGGED = {
    "periodic_disk_random": spec(150, 45, tau=0.65, disk=(70.3, 21.6, 9.2),
                                 si=W.disk_si_points(70.3, 21.6, 9.2, 72),
                                 init=("fields",) + random_fields(150, 45, 3)),
    "inlet_outlet_freeslip_naca": None,  # filled below
    "couette_walls_force": spec(131, 37, tau=0.8, eta=1e-3, edges=((P, 0, 0), (P, 0, 0), (V_, 0, 0), (V_, 0.02, 0)),
                                gx=1e-6, gy=-2e-7, disk=(40.0, 18.0, 6.0),
                                init=("fields",) + random_fields(131, 37, 5, amp=0.01)),
    "channel_walls_outflow_south": spec(67, 141, tau=0.6, edges=((V_, 0, 0), (V_, 0, 0), (OUT, 0, 0), (V_, 0, -0.01)),
                                        disk=(33.0, 100.0, 7.5), si=W.disk_si_points(33.0, 100.0, 7.5, 48),
                                        init=("uniform", 1.0, 0.0, -0.01)),
    "freeslip_west_east": spec(70, 90, tau=0.75, edges=((F, 0, 0), (F, 0, 0), (V_, 0, 0.02), (OUT, 0, 0)),
                               disk=(35.0, 45.0, 8.0), init=("uniform", 1.0, 0.0, 0.02)),
    "tiny_4x4": spec(4, 4, tau=0.9, eta=math.inf, init=("fields",) + random_fields(4, 4, 9)),
    "eta_inf_virtual_contour": spec(96, 70, tau=0.7, eta=math.inf, disk=(47.7, 33.1, 11.3),
                                    si=W.disk_si_points(47.7, 33.1, 11.3, 64),
                                    init=("fields",) + random_fields(96, 70, 13)),
}
_poly, _ref, _si = small_naca()
RAGGED["inlet_outlet_freeslip_naca"] = spec(150, 75, tau=0.56, edges=((V_, 0.05, 0), (OUT, 0, 0), (F, 0, 0), (F, 0, 0)),
                                            polygon=_poly, ref=_ref, si=_si, init=("uniform", 1.0, 0.05, 0.0))
RAGGED["trt_naca_paper_lambda"] = spec(150, 75, tau=0.55, trt=1.0 / 6.0,
                                      edges=((V_, 0.05, 0), (OUT, 0, 0), (F, 0, 0), (F, 0, 0)),
                                      polygon=_poly, ref=_ref, si=_si, init=("uniform", 1.0, 0.05, 0.0))
RAGGED["trt_walls_force_random"] = spec(133, 41, tau=0.7, eta=1e-3, trt=3.0 / 16.0,
                                       edges=((P, 0, 0), (P, 0, 0), (V_, 0, 0), (V_, 0.01, 0)), gx=2e-6,
                                       disk=(60.2, 20.7, 7.4), si=W.disk_si_points(60.2, 20.7, 7.4, 40),
                                       init=("fields",) + random_fields(133, 41, 23, amp=0.02))
RAGGED["si_interpolated_disk_random"] = spec(150, 45, tau=0.65, si_rule=1, disk=(70.3, 21.6, 9.2),
                                             si=W.disk_si_points(70.3, 21.6, 9.2, 72),
                                             init=("fields",) + random_fields(150, 45, 3))
RAGGED["si_interpolated_naca"] = spec(150, 75, tau=0.56, si_rule=1,
                                      edges=((V_, 0.05, 0), (OUT, 0, 0), (F, 0, 0), (F, 0, 0)),
                                      polygon=_poly, ref=_ref, si=_si, init=("uniform", 1.0, 0.05, 0.0))
RAGGED["convective_east_disk"] = spec(150, 45, tau=0.6, edges=((V_, 0.05, 0), (CV, 0.05, 0), (F, 0, 0), (F, 0, 0)),
                                     disk=(60.3, 21.6, 8.2), si=W.disk_si_points(60.3, 21.6, 8.2, 64),
                                     init=("fields",) + tuple(np.asarray(v) + (0.05 if k == 1 else 0.0) for k, v in
                                                             enumerate(random_fields(150, 45, 31, amp=0.01))))
RAGGED["convective_north_velocity_south"] = spec(70, 90, tau=0.75, edges=((F, 0, 0), (F, 0, 0), (V_, 0, 0.02),
                                                                         (CV, 0.02, 0)),
                                                 disk=(35.0, 45.0, 8.0), init=("uniform", 1.0, 0.0, 0.02))
RAGGED["convective_east_and_north_corner"] = spec(67, 53, tau=0.65, edges=((V_, 0.03, 0.01), (CV, 0.04, 0), (V_, 0, 0),
                                                                          (CV, 0.3, 0)),
                                                  disk=(30.2, 25.1, 6.3),
                                                  init=("fields",) + random_fields(67, 53, 41, amp=0.02))
RAGGED["convective_trt_naca"] = spec(150, 75, tau=0.55, trt=1.0 / 6.0,
                                     edges=((V_, 0.05, 0), (CV, 0.05, 0), (F, 0, 0), (F, 0, 0)),
                                     polygon=_poly, ref=_ref, si=_si, init=("uniform", 1.0, 0.05, 0.0))
_m = np.zeros((45, 77), np.uint8)
_m[0:6, :] = 1
_m[20:30, 10:14] = 1
_m[38:45, 60:77] = 1
_m[40:45, 0:5] = 1
RAGGED["host_mask_touching_periodic_edges"] = spec(77, 45, tau=0.7, eta=1e-2, mask=_m,
                                                   init=("fields",) + random_fields(77, 45, 17))


@pytest.mark.parametrize("name", sorted(RAGGED))
def test_ragged_cases_fp64(name):
    s = RAGGED[name]
    say(name, f"{s['nx']}x{s['ny']}")
    g = build_gpu(s, "f64")
    o = build_oracle(s)
    # solid indicator: bit-exact
    assert np.array_equal(g.mask() & 1, o.solid), name
    for k in range(3):
        g.step(20)
        o.step(20)
        compare_fp64(g, o, f"{name} after {20 * (k + 1)}")
    if o.si_node is not None:
        sample = np.zeros(o.nx * o.ny, bool)
        sample[o.si_node] = True
        assert np.array_equal((g.mask().ravel() & 0x40) != 0, sample), name


@pytest.mark.parametrize("source,rule", [(0, 0), (1, 0), (1, 1)])
def test_free_disk_sedimentation_fp64(source, rule):
    import dataclasses
    case = W.case_sedimentation(nx=80, ny=200, d=12.0, g=2e-4, y0=150.0, steps=300, npts=48,
                                force_source=source)
    case = dataclasses.replace(case, si_rule=rule)
    say("sedimentation 80x200 fp64 source", source, "si rule", rule)
    from gpu_cases import O
    from paper_2110_00967_amd import vplbm as V
    o = O.RefLattice.from_case(case)
    g = V.Lattice.from_case(case, precision="f64")
    for k in range(3):
        g.step(100)
        o.step(100)
        bg, bo = g.body_state(), o.body_state()
        assert np.abs(bg - bo).max() <= 1e-10 * max(1.0, np.abs(bo).max()), (k, bg, bo)
        assert np.array_equal(g.mask() & 1, o.solid)
    compare_fp64(g, o, f"sedimentation source {source}")
    assert o.body.y < 150.0 - 1.0  # it fell more than a cell


def test_prescribed_motion_galilean_fp64():
    U = (0.03, 0.02)
    s = spec(64, 48, tau=0.7, disk=(20.0, 20.0, 7.0), si=W.disk_si_points(20.0, 20.0, 7.0, 96),
             motion=(20.0, 20.0, 0.0, U[0], U[1], 0.0), init=("uniform", 1.0, U[0], U[1]))
    say("prescribed motion 64x48")
    g = build_gpu(s)
    o = build_oracle(s)
    g.step(60)
    o.step(60)
    compare_fp64(g, o, "galilean")
    assert np.abs(g.history(0)).max() <= 1e-13 and np.abs(g.history(1)).max() <= 1e-13
    assert abs(g.body_state()[0] - (20.0 + 60 * U[0])) < 1e-12


@pytest.mark.parametrize("npts,rule", [(1000, 0), (300, 1)])
def test_rotating_translating_disk_many_points_fp64(npts, rule):
    # a spinning, translating disk with many points: the sample selection
    # after each move sorts more than 256 keys (bitonic network) and, with
    # 1000 points, reads the points beyond its LDS staging from memory
    U, om = (0.02, -0.015), 0.01
    s = spec(96, 80, tau=0.68, eta=1e-3, disk=(40.0, 44.0, 12.5), si_rule=rule,
             si=W.disk_si_points(40.0, 44.0, 12.5, npts), motion=(40.0, 44.0, 0.3, U[0], U[1], om),
             init=("fields",) + random_fields(96, 80, 29, amp=0.01))
    say(f"rotating disk 96x80 fp64, {npts} points, rule {rule}")
    g = build_gpu(s)
    o = build_oracle(s)
    for k in range(3):
        g.step(15)
        o.step(15)
        compare_fp64(g, o, f"rotating disk after {g.step_count}")
        sample = np.zeros(o.nx * o.ny, bool)
        sample[o.si_node] = True
        assert np.array_equal((g.mask().ravel() & 0x40) != 0, sample)
    assert np.abs(g.body_state()[2] - (0.3 + 45 * om)) < 1e-12


@pytest.mark.parametrize("rule", [0, 1])
def test_si_at_matches_registered_points(rule):
    import dataclasses
    case = dataclasses.replace(W.case_disk_channel(steps=200), si_rule=rule)
    say("forces_si_at on the disk channel, si rule", rule)
    from gpu_cases import O
    from paper_2110_00967_amd import vplbm as V
    g = V.Lattice.from_case(case, precision="f64")
    g.step(200)
    once = g.forces_si_at(case.si_xy, case.si_n, case.si_ds)
    g.step(1)
    assert np.abs(once - g.forces_si()).max() <= 1e-12 * np.abs(once).max()


def test_fp32_disk_channel_accuracy():
    case = W.case_disk_channel()
    say("disk channel fp32 vs fp64 oracle")
    from gpu_cases import O
    from paper_2110_00967_amd import vplbm as V
    o = O.RefLattice.from_case(case)
    g = V.Lattice.from_case(case, precision="f32")
    g.step(case.steps, macro=True)
    o.step(case.steps)
    r, u, v = g.macro()
    err_u = rel_l2(np.stack([u, v]), np.stack([o.ux, o.uy]))
    q = 0.5 * case.u_ref ** 2 * case.length_scale
    me, si = g.forces_me() / q, g.forces_si() / q
    me_o, si_o = o.me()[-1] / q, o.si()[-1] / q
    say(f"fp32 u relL2={err_u:.2e} CD_ME {me[0]:.6f}/{me_o[0]:.6f} CD_SI {si[0]:.6f}/{si_o[0]:.6f}")
    assert err_u <= 1e-5
    assert abs(me[0] - me_o[0]) <= 0.005 * abs(me_o[0])
    assert abs(si[0] - si_o[0]) <= 0.005 * abs(si_o[0])
    assert abs(me[1] - me_o[1]) <= 0.005 * abs(me_o[0])
    assert abs(si[1] - si_o[1]) <= 0.005 * abs(si_o[0])


def test_fp16dev_disk_channel_reported():
    case = W.case_disk_channel()
    say("disk channel fp16dev vs fp64 oracle")
    from gpu_cases import O
    from paper_2110_00967_amd import vplbm as V
    o = O.RefLattice.from_case(case)
    g = V.Lattice.from_case(case, precision="f16dev")
    g.step(case.steps, macro=True)
    o.step(case.steps)
    r, u, v = g.macro()
    err_u = rel_l2(np.stack([u, v]), np.stack([o.ux, o.uy]))
    q = 0.5 * case.u_ref ** 2 * case.length_scale
    e_me = abs(g.forces_me()[0] - o.me()[-1][0]) / abs(o.me()[-1][0])
    e_si = abs(g.forces_si()[0] - o.si()[-1][0]) / abs(o.si()[-1][0])
    say(f"fp16dev u relL2={err_u:.2e} CD_ME rel err {e_me:.2e} CD_SI rel err {e_si:.2e}")
    assert np.isfinite(err_u) and err_u < 0.05  # reported figure; sanity bound only


def test_determinism_bitwise():
    case = W.case_disk_channel(steps=300)
    say("determinism fp32 x2")
    from paper_2110_00967_amd import vplbm as V
    runs = []
    for _ in range(2):
        g = V.Lattice.from_case(case, precision="f32")
        g.step(case.steps)
        runs.append((g.populations(), g.history(0), g.history(1)))
        g.close()
    for a, b in zip(*runs):
        assert np.array_equal(a, b)


def test_error_paths_on_device():
    from paper_2110_00967_amd import vplbm as V
    say("error paths")
    p = V.make_params(64, 32, 0.7, 1e-4, precision="f32")
    g = V.Lattice(p)
    with pytest.raises(V.VplbmError) as e:
        g.forces_me()
    assert e.value.code == V.ESTATE
    with pytest.raises(V.VplbmError) as e:
        g.macro()
    assert e.value.code == V.ESTATE
    with pytest.raises(V.VplbmError) as e:
        g.set_disk(2.0, 16.0, 5.0)  # touches the edge
    assert e.value.code == V.EINVAL
    g.set_disk(32.0, 16.0, 5.0)
    with pytest.raises(V.VplbmError) as e:
        # a point deep inside the disk with the normal pointing inwards: no fluid node
        g.set_si_points(np.array([[32.0, 16.0]]), np.array([[1.0, 0.0]]), np.array([1.0]))
    assert e.value.code == V.ENOSAMPLE
    with pytest.raises(V.VplbmError) as e:
        g.set_dynamics(-1.0, 0.0, 0.0)
    assert e.value.code == V.EINVAL
    g.init_uniform(1.0, 0.01, 0.0)
    g.step(3)
    g.sync()
    with pytest.raises(V.VplbmError) as e:
        g.force_history(0, 2, 5)  # beyond the last step
    assert e.value.code == V.EINVAL
    assert g.step_count == 3
