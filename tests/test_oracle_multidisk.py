"""The oracle's several-moving-disk mode, pinned by locality.

A lattice Boltzmann step moves information one cell per step, so two disks
more than 2 N cells apart cannot feel each other within N steps: each must
then move exactly as if it were alone.  The multi-disk bookkeeping (body ids
in the mask, per-body point frames and placement, per-body Newton-Euler
updates of Eqs. dep1 and theta2) is checked against the single-disk
oracle, itself pinned by the sedimentation, rotation and hydrostatic tests.
The lone disk's first step uses its points as given, the multi-disk mode
places them from the disk's frame (as every later step of both does), which
can round a coordinate one unit in the last place the other way; the bars
are 1e-12 (relative to the largest value), far below what a wrong body id,
frame or force assignment gives (1e-3 or more)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

NX, NY, STEPS = 120, 48, 20
TAU, ETA, G = 0.7, 1e-4, (0.0, -3e-5)
FREE = (24.3, 23.7, 6.2, 0.0, 0.0, 0.0, 0.0, 1.4)            # x, y, r, theta, u, v, omega, rho_s
SPUN = (92.1, 24.4, 5.1, 0.2, 0.004, -0.002, 0.01, 0.0)      # prescribed: moves by its velocities


def close(got, want):
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def points(d, n):
    return W.disk_si_points(d[0], d[1], d[2], n)


def lone(d, npts, source, rule):
    o = O.RefLattice(NX, NY, TAU, ETA, si_rule=rule)
    o.set_disk(d[0], d[1], d[2])
    o.set_si_points(*points(d, npts))
    if d[7] > 0:
        o.set_dynamics(d[7], *G, source)
    else:
        o.set_motion(d[0], d[1], d[3], d[4], d[5], d[6])
    o.init_uniform(1.0, 0.0, 0.0)
    o.step(STEPS)
    return o


@pytest.mark.parametrize("source,rule", [(0, 0), (1, 1)])
def test_far_disks_move_as_if_alone(source, rule):
    o = O.RefLattice(NX, NY, TAU, ETA, si_rule=rule)
    o.set_moving_disks([FREE, SPUN], *G, source)
    o.set_si_points_body(1, *points(FREE, 40))
    o.set_si_points_body(2, *points(SPUN, 32))
    o.init_uniform(1.0, 0.0, 0.0)
    o.step(STEPS)
    for body, d, n in ((1, FREE, 40), (2, SPUN, 32)):
        a = lone(d, n, source, rule)
        close(o.body_state(body), a.body_state(1))
        close(o.me(body), a.me(1))
        close(o.si(body), a.si(1))
        x0 = int(d[0]) - 12
        box = (slice(12, 36), slice(x0, x0 + 24))
        close(o.ft[box], a.ft[box])
        np.testing.assert_array_equal(o.solid[box] != 0, a.solid[box] != 0)
        assert set(np.unique(o.solid[box])) <= {0, body}
    # the free disk fell, the prescribed one moved by its velocities
    assert o.body_state(1)[4] < 0.0
    np.testing.assert_allclose(o.body_state(2)[:3], [SPUN[0] + STEPS * SPUN[4], SPUN[1] + STEPS * SPUN[5],
                                                     SPUN[3] + STEPS * SPUN[6]], rtol=0, atol=1e-12)


def test_overlap_takes_the_lower_id():
    o = O.RefLattice(40, 40, TAU, ETA)
    o.set_moving_disks([(18.0, 20.0, 5.0, 0, 0, 0, 0, 0), (24.0, 20.0, 5.0, 0, 0, 0, 0, 0)])
    one = O.mask_disk(40, 40, 18.0, 20.0, 5.0) != 0
    two = O.mask_disk(40, 40, 24.0, 20.0, 5.0) != 0
    assert (one & two).any()
    np.testing.assert_array_equal(o.solid == 1, one)
    np.testing.assert_array_equal(o.solid == 2, two & ~one)
