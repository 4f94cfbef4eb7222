"""Several static bodies in one lattice (body ids in mask bits 0-5), forces
per body, against the oracle.  FP64 bars as in test_gpu_parity: populations
within 1e-12, each body's force histories within 1e-10 of its largest
force; body ids and sample nodes bit-exact."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_cases import say

pytestmark = pytest.mark.gpu

NX, NY = 96, 48


def scene():
    ids = np.zeros((NY, NX), np.uint8)
    ids[O.mask_disk(NX, NY, 20.3, 24.2, 6.1) != 0] = 1
    ids[O.mask_disk(NX, NY, 47.1, 14.7, 4.9) != 0] = 2
    poly = np.array([[62.2, 25.1], [80.7, 27.3], [74.4, 38.8], [61.6, 34.2]])
    ids[O.mask_polygon(NX, NY, poly) != 0] = 3
    refs = [(20.3, 24.2), (47.1, 14.7), (69.0, 31.0)]
    pts = {1: W.disk_si_points(20.3, 24.2, 6.1, 44), 2: W.disk_si_points(47.1, 14.7, 4.9, 36),
           3: W.polygon_si_points(poly)}
    return ids, refs, pts


def fields(seed):
    ux, uy = W.smooth_random_velocity(NX, NY, seed=seed, amp=0.02)
    return W.random_density(NX, NY, seed=seed + 1, amp=1e-3), 0.03 + ux, uy


EDGES = ((O.VELOCITY, 0.03, 0.0), (O.OUTFLOW, 0, 0), (O.FREESLIP, 0, 0), (O.FREESLIP, 0, 0))


def build(precision="f64", tau=0.65, trt=0.0, edges=EDGES, seed=11):
    from paper_2110_00967_amd import vplbm as V
    ids, refs, pts = scene()
    p = V.make_params(NX, NY, tau, 1e-3, 1.0, precision, *edges, max_si_points=256, trt_lambda=trt,
                      max_bodies=4)
    g = V.Lattice(p)
    g.set_body_ids(ids, refs)
    for b, (xy, n, ds) in pts.items():
        g.set_si_points_body(b, xy, n, ds)
    g.set_fields(*fields(seed))
    o = O.RefLattice(NX, NY, tau, 1e-3, 1.0, *edges, trt_lambda=trt)
    o.set_body_ids(ids, refs)
    for b, (xy, n, ds) in pts.items():
        o.set_si_points_body(b, xy, n, ds)
    o.set_fields(*fields(seed))
    return g, o, ids


@pytest.mark.parametrize("trt", [0.0, 3.0 / 16.0])
def test_three_bodies_fp64_against_oracle(trt):
    from gpu_cases import oracle_pops
    from paper_2110_00967_amd import vplbm as V
    say("three static bodies 96x48 fp64, TRT" if trt else "three static bodies 96x48 fp64")
    g, o, ids = build(trt=trt)
    m = g.mask()
    assert np.array_equal(m & 0x3F, ids)
    sample = np.zeros(NX * NY, bool)
    sample[o.si_node] = True
    assert np.array_equal((m.ravel() & 0x40) != 0, sample)
    for _ in range(3):
        g.step(20)
        o.step(20)
        assert np.abs(g.populations() - oracle_pops(o)).max() <= 1e-12
    for b in (1, 2, 3):
        for which, ref in ((V.FORCE_ME, o.me(b)), (V.FORCE_SI, o.si(b))):
            h = g.history(which, body=b)
            e = np.abs(h - ref).max() / np.abs(ref).max()
            assert e <= 1e-10, (b, which, e)
        last = g.forces_body(b, V.FORCE_ME)
        assert np.abs(last - o.me(b)[-1]).max() <= 1e-10 * np.abs(o.me(b)).max()
    # body 1 through the single-body calls
    assert np.array_equal(g.forces_me(), g.forces_body(1, V.FORCE_ME))


def test_bodies_too_close_are_rejected():
    from paper_2110_00967_amd import vplbm as V
    say("bodies one cell apart")
    p = V.make_params(40, 20, 0.7, 1e-3, 1.0, "f32", max_bodies=2)
    g = V.Lattice(p)
    ids = np.zeros((20, 40), np.uint8)
    ids[5:10, 5:10] = 1
    ids[5:10, 11:15] = 2  # column 10 is fluid and linked to both
    with pytest.raises(V.VplbmError) as e:
        g.set_body_ids(ids, [(7, 7), (12, 7)])
    assert e.value.code == V.EINVAL
    ids[5:10, 11:15] = 0
    ids[5:10, 12:15] = 2  # two fluid columns between them: fine
    g.set_body_ids(ids, [(7, 7), (13, 7)])
    with pytest.raises(V.VplbmError):
        g.set_body_ids(ids, [(7, 7)])  # id 2 > nbody


def test_multibody_in_batch_equals_alone():
    from paper_2110_00967_amd import vplbm as V
    say("multi-body lattice inside a batch, fp32")
    g, _, _ = build("f32")
    for _ in range(37):  # plain per-step launches
        g.step(1)
    alone = [g.history(w, body=b) for b in (1, 2, 3) for w in (V.FORCE_ME, V.FORCE_SI)]
    pops = g.populations()
    g.close()
    a, _, _ = build("f32")
    other = V.Lattice.from_case(W.case_disk_channel(), precision="f32")
    bt = V.Batch([other, a])
    bt.step([20, 37])
    assert np.array_equal(a.populations(), pops)
    got = [a.history(w, body=b) for b in (1, 2, 3) for w in (V.FORCE_ME, V.FORCE_SI)]
    for x, y in zip(got, alone):
        assert np.array_equal(x, y)
    bt.close()


def test_forces_do_not_depend_on_the_tile():
    # ME is summed per interface cell and SI per sample record, in an order
    # fixed at set-up: every tile shape gives the same bits
    from paper_2110_00967_amd import vplbm as V
    say("tile shapes 64x4 / 128x2 / 256x1 / 64x1, three bodies fp32")
    runs = []
    for bx, by in ((64, 4), (128, 2), (256, 1), (64, 1)):
        g, _, _ = build("f32", trt=3.0 / 16.0)
        g.set_tile(bx, by)
        g.step(25)
        runs.append([g.populations()] + [g.history(w, body=b) for b in (1, 2, 3)
                                         for w in (V.FORCE_ME, V.FORCE_SI)])
        g.close()
    for r in runs[1:]:
        for a, b in zip(r, runs[0]):
            assert np.array_equal(a, b)


def test_interface_slot_capacity():
    from paper_2110_00967_amd import vplbm as V
    say("interface slot capacity")
    g = V.Lattice(V.make_params(96, 48, 0.65, 1e-3, 1.0, "f32", max_interface_cells=20))
    with pytest.raises(V.VplbmError) as e:
        g.set_disk(40.0, 24.0, 8.0)  # about 60 interface cells
    assert e.value.code == V.EINVAL
    g.close()
    # a moving disk keeps per-tile force sums in these slots: its points at
    # radius 39.5 give a window half size h = 40 + 8, 97 cells a side, which can
    # meet (ceil(96 / 64) + 1) x (ceil(96 / 4) + 1) = 3 x 25 tiles of 64 x 4;
    # 8 doubles a tile, 150 slots of 4 (the disk alone has 52 interface cells)
    th = np.arange(64) * (2 * np.pi / 64)
    xy = np.stack([64 + 39.5 * np.cos(th), 64 + 39.5 * np.sin(th)], 1)
    nrm = np.stack([np.cos(th), np.sin(th)], 1)
    ds = np.full(64, 2 * np.pi * 39.5 / 64)

    def lattice(cap):
        g = V.Lattice(V.make_params(128, 128, 0.65, 1e-3, 1.0, "f32", max_interface_cells=cap,
                                    max_si_points=64))
        g.set_disk(64.0, 64.0, 3.0)
        g.set_si_points(xy, nrm, ds)
        return g

    g = lattice(149)
    with pytest.raises(V.VplbmError) as e:
        g.set_motion(64.0, 64.0, 0.0, 0.01, 0.0, 0.0)
    assert e.value.code == V.EINVAL
    g.close()
    g = lattice(150)
    g.set_motion(64.0, 64.0, 0.0, 0.01, 0.0, 0.0)
    g.init_uniform(1.0, 0.0, 0.0)
    g.step(40)
    g.sync()
    assert np.isfinite(g.forces_me()).all()
    g.close()


# -- several moving disks ------------------------------------------------------
MOVING = [(30.2, 36.1, 6.1, 0.0, 0.0, 0.0, 0.0, 1.3),          # free
          (64.4, 20.3, 5.2, 0.0, 0.0, 0.0, 0.0, 1.8),          # free, heavier
          (96.3, 47.8, 5.6, 0.1, -0.004, 0.003, 0.008, 0.0)]   # prescribed: translating and spinning
MEDGES = ((O.VELOCITY, 0.02, 0.0), (O.OUTFLOW, 0, 0), (O.FREESLIP, 0, 0), (O.FREESLIP, 0, 0))
MNX, MNY, MG = 128, 72, (0.0, -2e-5)


def moving_build(precision="f64", source=0, rule=0):
    from paper_2110_00967_amd import vplbm as V
    p = V.make_params(MNX, MNY, 0.7, 1e-4, 1.0, precision, *MEDGES, max_si_points=256, si_rule=rule,
                      max_bodies=3)
    g = V.Lattice(p)
    g.set_moving_disks(MOVING, *MG, source)
    o = O.RefLattice(MNX, MNY, 0.7, 1e-4, 1.0, *MEDGES, si_rule=rule)
    o.set_moving_disks(MOVING, *MG, source)
    for b, d, n in ((1, MOVING[0], 40), (2, MOVING[1], 32), (3, MOVING[2], 36)):
        pts = W.disk_si_points(d[0], d[1], d[2], n)
        g.set_si_points_body(b, *pts)
        o.set_si_points_body(b, *pts)
    g.init_uniform(1.0, 0.02, 0.0)
    o.init_uniform(1.0, 0.02, 0.0)
    return g, o


@pytest.mark.parametrize("source,rule", [(0, 0), (1, 1)])
def test_moving_disks_fp64_against_oracle(source, rule):
    from gpu_cases import oracle_pops
    from paper_2110_00967_amd import vplbm as V
    say(f"three moving disks {MNX}x{MNY} fp64, source {source}, rule {rule}")
    g, o = moving_build("f64", source, rule)
    assert np.array_equal(g.mask() & 0x3F, o.solid)
    for k in range(3):
        g.step(50)
        o.step(50)
        assert np.abs(g.populations() - oracle_pops(o)).max() <= 1e-12, k
        for b in (1, 2, 3):
            bg, bo = g.body_state(b), o.body_state(b)
            assert np.abs(bg - bo).max() <= 1e-10 * max(1.0, np.abs(bo).max()), (k, b, bg, bo)
        m = g.mask()
        assert np.array_equal(m & 0x3F, o.solid), k
        sample = np.zeros(MNX * MNY, bool)
        sample[o.si_node] = True
        assert np.array_equal((m.ravel() & 0x40) != 0, sample), k
    for b in (1, 2, 3):
        for which, ref in ((V.FORCE_ME, o.me(b)), (V.FORCE_SI, o.si(b))):
            e = np.abs(g.history(which, body=b) - ref).max() / np.abs(ref).max()
            assert e <= 1e-10, (b, which, e)
    # the free disks moved on their own forces; the prescribed one by its velocities
    assert abs(o.body_state(1)[4]) > 1e-5 and abs(o.body_state(2)[4]) > 1e-5
    assert abs(g.body_state(3)[0] - (MOVING[2][0] + 150 * MOVING[2][4])) < 1e-10


def test_moving_disks_in_batch_equal_alone():
    from paper_2110_00967_amd import vplbm as V
    say("three moving disks inside a batch, fp32")
    g, _ = moving_build("f32")
    for _ in range(29):
        g.step(1)
    alone = [g.history(w, body=b) for b in (1, 2, 3) for w in (V.FORCE_ME, V.FORCE_SI)]
    states = [g.body_state(b) for b in (1, 2, 3)]
    pops = g.populations()
    g.close()
    a, _ = moving_build("f32")
    other = V.Lattice.from_case(W.case_disk_channel(), precision="f32")
    bt = V.Batch([other, a])
    bt.step([11, 29])
    assert np.array_equal(a.populations(), pops)
    for x, y in zip([a.history(w, body=b) for b in (1, 2, 3) for w in (V.FORCE_ME, V.FORCE_SI)], alone):
        assert np.array_equal(x, y)
    for b in (1, 2, 3):
        assert np.array_equal(a.body_state(b), states[b - 1])
    bt.close()


@pytest.mark.parametrize("big", [False, True])
def test_several_lattices_with_moving_disks_in_one_batch(big):
    # three lattices with moving disks (three disks; one sedimenting disk
    # driven by SI; one by ME) and a static one, stepped different counts by
    # one batch: every lattice as alone, bit for bit.  The batch's launches
    # start their XCD bands at the disks' hit boxes (below 8192 tiles of
    # 64x4); with a large static lattice added (big) they run the form
    # without rotation until the last chunk, whose two lattices fall below
    # the limit again
    from paper_2110_00967_amd import vplbm as V
    say(f"several lattices with moving disks in one batch, fp32, big={big}")

    def build():
        a, _ = moving_build("f32")
        c1 = W.case_sedimentation()
        c2 = W.case_sedimentation()
        c2.force_source = V.FORCE_SI if c1.force_source == V.FORCE_ME else V.FORCE_ME
        lats = [a, V.Lattice.from_case(c1, precision="f32"), V.Lattice.from_case(W.case_disk_channel(),
                precision="f32"), V.Lattice.from_case(c2, precision="f32")]
        if big:
            g = V.Lattice(V.make_params(1024, 512, 0.6, 1e-4, 1.0, "f32"))
            g.init_uniform(1.0, 0.04, 0.01)
            lats.append(g)
        return lats

    nsteps = [29, 40, 11, 35] + ([38] if big else [])
    alone = build()
    for g, n in zip(alone, nsteps):
        for _ in range(n):
            g.step(1)
    lats = build()
    if big:
        def tiles(g):
            return -(-g.nx // 64) * -(-g.ny // 4)
        # chunks of all five, four and three lattices above the limit, the
        # last two (c1 and the static lattice, then c1) below it
        assert sum(tiles(g) for g in lats if g is not lats[2]) - tiles(lats[0]) > 8192
        assert tiles(lats[1]) + tiles(lats[4]) < 8192
    bt = V.Batch(lats)
    bt.step(nsteps)
    nb = [3, 1, 1, 1, 0]
    for k, (g, r) in enumerate(zip(lats, alone)):
        assert g.step_count == r.step_count == nsteps[k]
        assert np.array_equal(g.populations(), r.populations()), k
        for b in range(1, nb[k] + 1):
            for w in (V.FORCE_ME, V.FORCE_SI):
                assert np.array_equal(g.history(w, body=b), r.history(w, body=b)), (k, b, w)
            if k != 2:
                assert np.array_equal(g.body_state(b), r.body_state(b)), (k, b)
    bt.close()
    for g in lats + alone:
        g.close()


def test_moving_disks_too_close_are_rejected():
    from paper_2110_00967_amd import vplbm as V
    say("moving disks one cell apart")
    g = V.Lattice(V.make_params(64, 40, 0.7, 1e-3, 1.0, "f32", max_bodies=2))
    with pytest.raises(V.VplbmError) as e:
        g.set_moving_disks([(20.0, 20.0, 5.0, 0, 0, 0, 0, 1.2), (31.5, 20.0, 5.0, 0, 0, 0, 0, 1.2)])
    assert e.value.code == V.EINVAL
    g.set_moving_disks([(20.0, 20.0, 5.0, 0, 0, 0, 0, 1.2), (32.5, 20.0, 5.0, 0, 0, 0, 0, 1.2)])
    with pytest.raises(V.VplbmError):
        g.set_moving_disks([(20.0, 20.0, 5.0, 0, 0, 0, 0, 1.2)] * 3)  # more than max_bodies


# -- static bodies on non-periodic edges ----------------------------------------
def test_bodies_on_walls_fp64():
    # bodies whose cells lie on the south and north walls: a fluid cell on a
    # wall takes its links' body from its own side, never from the solid
    # cells across the wall (no neighbours there)
    from gpu_cases import oracle_pops
    from paper_2110_00967_amd import vplbm as V
    nx, ny = 64, 40
    edges = ((O.VELOCITY, 0.03, 0.0), (O.OUTFLOW, 0, 0), (O.FREESLIP, 0, 0), (O.VELOCITY, 0.0, 0.0))
    ids = np.zeros((ny, nx), np.uint8)
    ids[0:6, 20:30] = 1                      # on the south wall
    ids[35:40, 16:34] = 2                    # on the north wall, over body 1 across the wrap
    ids[O.mask_disk(nx, ny, 46.2, 20.4, 5.3) != 0] = 3
    refs = [(24.5, 2.5), (24.5, 37.5), (46.2, 20.4)]
    say("three static bodies on the walls 64x40 fp64")
    p = V.make_params(nx, ny, 0.7, 1e-3, 1.0, "f64", *edges, max_si_points=64, max_bodies=3)
    g = V.Lattice(p)
    g.set_body_ids(ids, refs)
    o = O.RefLattice(nx, ny, 0.7, 1e-3, 1.0, *edges)
    o.set_body_ids(ids, refs)
    pts = W.disk_si_points(46.2, 20.4, 5.3, 36)
    g.set_si_points_body(3, *pts)
    o.set_si_points_body(3, *pts)
    rho, ux, uy = W.random_density(nx, ny, seed=5, amp=1e-3), *W.smooth_random_velocity(nx, ny, seed=6, amp=0.02)
    g.set_fields(rho, ux, uy)
    o.set_fields(rho, ux, uy)
    for _ in range(3):
        g.step(20)
        o.step(20)
        assert np.abs(g.populations() - oracle_pops(o)).max() <= 1e-12
    for b in (1, 2, 3):
        for which, ref in ((V.FORCE_ME, o.me(b)), (V.FORCE_SI, o.si(b))):
            if not np.abs(ref).max():
                continue
            e = np.abs(g.history(which, body=b) - ref).max() / np.abs(ref).max()
            assert e <= 1e-10, (b, which, e)
