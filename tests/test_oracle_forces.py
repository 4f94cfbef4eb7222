"""Pins of the oracle's two force reductions (Sec. 2.3) and rigid-body update.

Momentum exchange (Eq. MMEL, its sum and Eq. fluidtorque):
  * momentum balance: for a body at rest, the momentum that streaming moves
    into the solid cells equals the link sum exactly, for any state;
  * the link form equals the per-destination ("pulled") form of the same
    exchange, also for a moving body (u_G and torque arms included);
  * zero force at rest, for a body-free uniform flow seen through a virtual
    contour, and for a disk moving with the flow (Galilean invariance);
  * mirror symmetry: the disk channel is symmetric about its mid row, so the
    lift and torque vanish.
Stress integration (Eq. defFf and the sigma definition):
  * Poiseuille: sigma_xy = rho0 nu du/dy = G/2 (ny - 1 - 2y) at any node;
  * Taylor-Green: deviatoric normal stress 2 rho nu du/dx and zero shear;
  * the same zero-force and symmetry cases as above.
Hydrostatics (a disk at rest in a closed box under a uniform force density):
  * stress integration gives the Archimedes force of the pressure part of
    sigma, -(rho - rho0) c_s^2 I, in closed form for the interpolated stencil
    and from the sample nodes' heights for the nearest-node rule;
  * momentum exchange balances the force density on the solid cells.
Rigid body (Eqs. dep1, theta2): closed forms of uniform acceleration; the
stress-integration points of a rotating, translating body follow the rigid
motion (a quarter turn maps them exactly, one step moves them with the body's
velocity field).
"""
import ctypes as C
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

CX, CY = O.CX, O.CY
OPP = [0, 3, 4, 1, 2, 7, 8, 5, 6]
MAGIC_TAU = 0.5 + math.sqrt(3.0 / 16.0)


def random_state(lat, seed, amp=0.03):
    ux, uy = W.smooth_random_velocity(lat.nx, lat.ny, seed=seed, amp=amp)
    rho = W.random_density(lat.nx, lat.ny, seed=seed + 1, amp=1e-3)
    lat.set_fields(rho, ux, uy)
    g = np.random.default_rng(seed + 2)
    lat.ft += 1e-4 * g.standard_normal(lat.ft.shape)  # off-equilibrium parts


def solid_momentum(f, solid):
    m = solid.astype(bool)
    return np.array([(f[m] * CX).sum(), (f[m] * CY).sum()])


def test_me_momentum_balance_identity():
    lat = O.RefLattice(40, 36, 0.7, 1e-4)
    lat.set_disk(19.4, 17.8, 7.3)
    random_state(lat, 21)
    for _ in range(3):
        before = solid_momentum(lat.ft, lat.solid)
        lat.step(1)
        after = solid_momentum(lat.streamed(), lat.solid)
        me = lat.me()[-1]
        assert np.abs((after - before) - me[:2]).max() <= 1e-14 * max(1.0, np.abs(me[:2]).max())


def pulled_form(lat, f_streamed, body):
    """Per-destination form of the exchange: at every node, every pulled
    population that crossed the solid/fluid boundary, signed by direction,
    with the link midpoint measured from the link's fluid node."""
    bx, by, th, bu, bv, bw = body
    solid = lat.solid
    ny, nx = solid.shape
    F = np.zeros(2)
    T = 0.0
    for y in range(ny):
        for x in range(nx):
            for a in range(1, 9):
                sx, sy = (x - CX[a]) % nx, (y - CY[a]) % ny
                if solid[y, x] == solid[sy, sx]:
                    continue
                if solid[y, x]:   # fluid -> solid: fluid node is the source
                    gx, gy, s = sx + 0.5 * CX[a], sy + 0.5 * CY[a], 1.0
                else:             # solid -> fluid: fluid node is this node
                    gx, gy, s = x - 0.5 * CX[a], y - 0.5 * CY[a], -1.0
                ugx, ugy = bu - bw * (gy - by), bv + bw * (gx - bx)
                lx = s * (CX[a] - ugx) * f_streamed[y, x, a]
                ly = s * (CY[a] - ugy) * f_streamed[y, x, a]
                F += (lx, ly)
                T += (gx - bx) * ly - (gy - by) * lx
    return np.array([F[0], F[1], T])


def test_me_link_form_equals_pulled_form_moving_body():
    lat = O.RefLattice(30, 26, 0.65, 1e-4)
    lat.set_disk(14.6, 12.2, 6.1)
    b = lat.body
    b.u, b.v, b.omega = 0.013, -0.007, 0.0021  # velocities only; mask stays
    random_state(lat, 31)
    body = lat.body_state().copy()
    lat.step(1)
    me = lat.me()[-1]
    ref = pulled_form(lat, lat.streamed(), body)
    assert np.abs(me - ref).max() <= 1e-14 * np.abs(ref).max()


def test_zero_force_at_rest():
    lat = O.RefLattice(40, 30, 0.8, 1e-4)
    lat.set_disk(20.0, 15.0, 6.0)
    xy, n, ds = W.disk_si_points(20.0, 15.0, 6.0, 64)
    lat.set_si_points(xy, n, ds)
    lat.init_uniform(1.0, 0.0, 0.0)
    f0 = lat.ft.copy()
    lat.step(20)
    # f^eq(1, 0) = w_a; only the rounding of sum(w) = 1 moves it
    assert np.abs(lat.ft - f0).max() <= 1e-15
    assert np.abs(lat.me()).max() <= 1e-15
    assert np.abs(lat.si()).max() <= 1e-15


def test_zero_force_body_free_uniform_flow():
    # eta = +inf: the disk only marks links and sample nodes (a virtual contour)
    U = (0.04, -0.015)
    lat = O.RefLattice(48, 40, 0.7, float("inf"))
    lat.set_disk(23.3, 19.6, 8.4)
    xy, n, ds = W.disk_si_points(23.3, 19.6, 8.4, 96)
    lat.set_si_points(xy, n, ds)
    one = np.ones((lat.ny, lat.nx))
    lat.set_fields(one, U[0] * one, U[1] * one)  # inside the contour too
    lat.step(10)
    assert np.abs(lat.me()).max() <= 1e-13
    assert np.abs(lat.si()).max() <= 1e-13


def test_zero_force_disk_moving_with_the_flow():
    U = (0.03, 0.02)
    lat = O.RefLattice(64, 48, 0.7, 1e-4)
    lat.set_disk(20.0, 20.0, 7.0)
    xy, n, ds = W.disk_si_points(20.0, 20.0, 7.0, 96)
    lat.set_si_points(xy, n, ds)
    lat.set_motion(20.0, 20.0, 0.0, U[0], U[1], 0.0)
    lat.init_uniform(1.0, *U)
    lat.step(60)  # the mask moves by more than a cell
    assert abs(lat.body.x - (20.0 + 60 * U[0])) < 1e-12
    assert np.abs(lat.me()).max() <= 1e-13
    assert np.abs(lat.si()).max() <= 1e-13


def test_disk_channel_mirror_symmetry():
    case = W.case_disk_channel(steps=600)
    lat = O.RefLattice.from_case(case)
    lat.step(case.steps)
    me, si = lat.me()[-1], lat.si()[-1]
    assert me[0] > 0 and si[0] > 0
    assert abs(me[1]) <= 1e-10 * me[0] and abs(si[1]) <= 1e-10 * si[0]
    assert abs(me[2]) <= 1e-10 * me[0] * 8 and abs(si[2]) <= 1e-10 * si[0] * 8


def test_si_poiseuille_shear():
    G, ny, nx = 1e-6, 16, 4
    nu = (MAGIC_TAU - 0.5) / 3
    lat = O.RefLattice(nx, ny, MAGIC_TAU, float("inf"), south=(O.VELOCITY, 0, 0), north=(O.VELOCITY, 0, 0), gx=G)
    y0 = 3
    xy = np.array([[x, y0] for x in range(nx)], float)
    n = np.tile([0.0, 1.0], (nx, 1))
    lat.set_si_points(xy, n, np.ones(nx))
    lat.init_uniform(1.0, 0.0, 0.0)
    lat.step(int(30 * ny * ny / nu))
    Fx = lat.si()[-1][0]
    assert abs(Fx - nx * G / 2 * (ny - 1 - 2 * y0)) <= 1e-9 * abs(Fx)
    # lower wall line, normal pointing down: the fluid pulls the wall along +x
    xy[:, 1] = 0
    n[:, 1] = -1.0
    lat.set_si_points(xy, n, np.ones(nx))
    lat.step(1)
    assert abs(lat.si()[-1][0] + nx * G / 2 * (ny - 1)) <= 1e-9 * nx * G * ny


def test_si_taylor_green_stress():
    L, tau, U0 = 64, 0.8, 0.01
    nu = (tau - 0.5) / 3
    k = 2 * math.pi / L
    x = np.arange(L)[None, :]
    y = np.arange(L)[:, None]
    p = -U0 ** 2 / 4 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    lat = O.RefLattice(L, L, tau, float("inf"))
    lat.set_fields(1 + 3 * p, -U0 * np.cos(k * x) * np.sin(k * y), U0 * np.sin(k * x) * np.cos(k * y))
    nsteps = 40
    lat.step(nsteps)
    f = lat.streamed()
    dec = math.exp(-2 * nu * k * k * nsteps)
    for (i, j) in [(5, 9), (13, 3), (40, 22)]:
        s = np.zeros(3)
        O.lib().orc_node_stress(C.byref(lat.p), np.ascontiguousarray(f[j, i]), s)
        dudx = U0 * dec * k * math.sin(k * i) * math.sin(k * j)
        assert abs(0.5 * (s[0] - s[2]) - 2 * nu * dudx) <= 0.02 * abs(2 * nu * dudx)
        assert abs(s[1]) <= 0.01 * abs(2 * nu * dudx) + 1e-9


def test_newton_euler_uniform_acceleration():
    b = O._Body()
    b.x, b.y = 5.0, 100.0
    rho_s, g = 1.5, -1e-4
    a = (1 - 1 / rho_s) * g
    for n in range(1, 200):
        O.lib().orc_body_update(C.byref(b), np.zeros(3), 10.0, 3.0, 1.0, rho_s, 0.0, g)
        # semi-implicit Euler: v_n = n a, y_n = y_0 + a n (n + 1) / 2
        assert abs(b.v - n * a) <= 1e-15 * n
        assert abs(b.y - (100.0 + a * n * (n + 1) / 2)) <= 1e-12
    assert b.x == 5.0 and b.u == 0.0 and b.omega == 0.0


def test_newton_euler_constant_force_and_torque():
    b = O._Body()
    m, inertia, F, T = 50.0, 120.0, 2e-3, -3e-4
    for n in range(1, 100):
        O.lib().orc_body_update(C.byref(b), np.array([F, 0.0, T]), m, inertia, 1.0, 2.0, 0.0, 0.0)
        assert abs(b.x - F / m * n * (n + 1) / 2) <= 1e-14
        assert abs(b.theta - T / inertia * n * (n + 1) / 2) <= 1e-14


# ---------------------------------------------------------------------------
# interpolated stress-integration stencil (rule 1)
# ---------------------------------------------------------------------------

def test_si_interpolated_poiseuille_shear_exact():
    # sigma_xy is linear in y: bilinear interpolation at p = x + 1.5 n is exact
    G, ny, nx = 1e-6, 16, 6
    nu = (MAGIC_TAU - 0.5) / 3
    lat = O.RefLattice(nx, ny, MAGIC_TAU, float("inf"), south=(O.VELOCITY, 0, 0), north=(O.VELOCITY, 0, 0),
                       gx=G, si_rule=1)
    y0 = 2.3
    xy = np.array([[x + 0.37, y0] for x in range(nx - 1)], float)
    n = np.tile([0.0, 1.0], (len(xy), 1))
    lat.set_si_points(xy, n, np.ones(len(xy)))
    assert (lat.si_node4.reshape(-1, 4) >= 0).all()  # every point interpolates
    lat.init_uniform(1.0, 0.0, 0.0)
    lat.step(int(30 * ny * ny / nu))
    yp = y0 + 1.5
    ref = len(xy) * G / 2 * (ny - 1 - 2 * yp)
    assert abs(lat.si()[-1][0] - ref) <= 1e-9 * abs(ref)


def test_si_interpolated_stencil_properties():
    nx = ny = 40
    xc, yc, r = 19.6, 20.3, 7.7
    solid = O.mask_disk(nx, ny, xc, yc, r)
    xy, n, ds = W.disk_si_points(xc, yc, r, 96)
    node4, w4, missing = O.si_stencils(solid, xy, n, rule=1)
    assert missing == 0
    node4, w4 = node4.reshape(-1, 4), w4.reshape(-1, 4)
    ninterp = 0
    for (px, py), (nx_, ny_), nd, w in zip(xy, n, node4, w4):
        used = nd >= 0
        assert abs(w.sum() - 1.0) <= 1e-14 and (w >= 0).all()
        assert all(solid[k // nx, k % nx] == 0 for k in nd[used])
        if used.sum() == 4:
            ninterp += 1
            qx, qy = px + 1.5 * nx_, py + 1.5 * ny_
            X, Y = nd % nx, nd // nx
            assert X.min() <= qx <= X.max() and Y.min() <= qy <= Y.max()
            # the weights reproduce p itself (bilinear interpolation of x and y)
            assert abs((w * X).sum() - qx) <= 1e-12 and abs((w * Y).sum() - qy) <= 1e-12
    assert ninterp >= 80  # most points clear the surface at 1.5 cells


def test_si_interpolated_zero_force_uniform_flow():
    U = (0.04, -0.015)
    lat = O.RefLattice(48, 40, 0.7, float("inf"), si_rule=1)
    lat.set_disk(23.3, 19.6, 8.4)
    xy, n, ds = W.disk_si_points(23.3, 19.6, 8.4, 96)
    lat.set_si_points(xy, n, ds)
    one = np.ones((lat.ny, lat.nx))
    lat.set_fields(one, U[0] * one, U[1] * one)
    lat.step(10)
    assert np.abs(lat.si()).max() <= 1e-13


# ----------------------------------------------------------------------------
# several bodies in one lattice: ids in the mask, forces per body
# ----------------------------------------------------------------------------

def three_bodies(nx=72, ny=40):
    ids = np.zeros((ny, nx), np.uint8)
    ids[O.mask_disk(nx, ny, 16.3, 20.2, 5.6) != 0] = 1
    ids[O.mask_disk(nx, ny, 38.1, 12.7, 4.4) != 0] = 2
    poly = np.array([[50.2, 22.1], [62.7, 24.3], [58.4, 33.8], [49.6, 30.2]])
    ids[O.mask_polygon(nx, ny, poly) != 0] = 3
    pts = {1: W.disk_si_points(16.3, 20.2, 5.6, 40), 2: W.disk_si_points(38.1, 12.7, 4.4, 32),
           3: W.polygon_si_points(poly)}
    return ids, pts


def multi_lattice(ids, refs, pts, seed=7, nx=72, ny=40):
    lat = O.RefLattice(nx, ny, 0.65, 1e-3, west=(O.VELOCITY, 0.03, 0), east=(O.OUTFLOW, 0, 0),
                       south=(O.FREESLIP, 0, 0), north=(O.FREESLIP, 0, 0))
    lat.set_body_ids(ids, refs)
    for b, (xy, n, ds) in pts.items():
        lat.set_si_points_body(b, xy, n, ds)
    random_state(lat, seed)
    return lat


def test_multibody_forces_add_up_to_the_union():
    ids, pts = three_bodies()
    Z = (40.0, 20.0)
    a = multi_lattice(ids, [Z] * 3, pts)
    allp = tuple(np.concatenate([pts[b][k] for b in (1, 2, 3)]) for k in range(3))
    b = multi_lattice((ids > 0).astype(np.uint8), [Z], {1: allp})
    a.step(12)
    b.step(12)
    me = sum(a.me(k) for k in (1, 2, 3))
    si = sum(a.si(k) for k in (1, 2, 3))
    assert np.abs(me - b.me(1)).max() <= 1e-13 * np.abs(b.me(1)).max()
    assert np.abs(si - b.si(1)).max() <= 1e-13 * np.abs(b.si(1)).max()
    assert np.abs(a.ft - b.ft).max() == 0.0  # attribution does not touch the flow


def test_multibody_torque_about_each_reference():
    # T about r_b = T about Z + (Z - r_b) x F, for both methods
    ids, pts = three_bodies()
    Z = (40.0, 20.0)
    refs = [(16.3, 20.2), (38.1, 12.7), (55.0, 27.0)]
    a = multi_lattice(ids, refs, pts)
    z = multi_lattice(ids, [Z] * 3, pts)
    a.step(6)
    z.step(6)
    for k, (rx, ry) in enumerate(refs, start=1):
        for ha, hz in ((a.me(k), z.me(k)), (a.si(k), z.si(k))):
            F = hz[:, :2]
            expect = hz[:, 2] + (Z[0] - rx) * F[:, 1] - (Z[1] - ry) * F[:, 0]
            assert np.abs(ha[:, :2] - F).max() <= 1e-15 * np.abs(F).max() + 1e-300
            assert np.abs(ha[:, 2] - expect).max() <= 1e-12 * np.abs(hz[:, 2]).max()


def test_multibody_first_step_me_ignores_other_bodies():
    # the ME of step 1 depends on the initial state only: body 1's value is
    # the one of the same state with body 1 alone
    ids, pts = three_bodies()
    refs = [(16.3, 20.2), (38.1, 12.7), (55.0, 27.0)]
    a = multi_lattice(ids, refs, pts)
    one = np.where(ids == 1, 1, 0).astype(np.uint8)
    b = multi_lattice(one, refs[:1], {1: pts[1]})
    a.step(1)
    b.step(1)
    assert np.abs(a.me(1) - b.me(1)).max() <= 1e-15 * np.abs(b.me(1)).max()
    assert np.abs(a.si(1) - b.si(1)).max() <= 1e-15 * np.abs(b.si(1)).max()


def test_multibody_mirror_twins():
    # two equal disks mirrored about the channel's mid-line in a symmetric
    # flow: equal drag, opposite lift and torque
    nx, ny = 64, 41
    yc = 20.0
    ids = np.zeros((ny, nx), np.uint8)
    ids[O.mask_disk(nx, ny, 20.0, yc + 7.0, 4.5) != 0] = 1
    ids[O.mask_disk(nx, ny, 20.0, yc - 7.0, 4.5) != 0] = 2
    lat = O.RefLattice(nx, ny, 0.7, 1e-3, west=(O.VELOCITY, 0.03, 0), east=(O.OUTFLOW, 0, 0),
                       south=(O.FREESLIP, 0, 0), north=(O.FREESLIP, 0, 0))
    lat.set_body_ids(ids, [(20.0, yc + 7.0), (20.0, yc - 7.0)])
    p1 = W.disk_si_points(20.0, yc + 7.0, 4.5, 36)
    xy2 = p1[0].copy()
    xy2[:, 1] = 2 * yc - xy2[:, 1]
    n2 = p1[1].copy()
    n2[:, 1] = -n2[:, 1]
    lat.set_si_points_body(1, *p1)
    lat.set_si_points_body(2, xy2, n2, p1[2])
    lat.init_uniform(1.0, 0.03, 0.0)
    lat.step(300)
    for h1, h2 in ((lat.me(1), lat.me(2)), (lat.si(1), lat.si(2))):
        scale = np.abs(h1).max()
        assert np.abs(h1[:, 0] - h2[:, 0]).max() <= 1e-12 * scale
        assert np.abs(h1[:, 1] + h2[:, 1]).max() <= 1e-12 * scale
        assert np.abs(h1[:, 2] + h2[:, 2]).max() <= 1e-12 * scale
    assert np.abs(lat.me(1)[-1, 1]) > 1e-3 * np.abs(lat.me(1)[-1, 0])  # a real lift to mirror


# ----------------------------------------------------------------------------
# hydrostatics: the pressure part of sigma and the momentum balance of ME
# ----------------------------------------------------------------------------

def hydrostatic_box(rule, L=32, g=2e-5, r=7.5, npts=64, steps=3000, eta=1e-4):
    """A penalized disk at rest in a closed box of fluid at rest under a
    uniform force density G = (0, -g).  The steady state is hydrostatic:
    u = 0 and c_s^2 grad rho = G, so rho falls linearly with height and the
    stress is the pressure alone, sigma = -(rho - rho0) c_s^2 I.  Started
    from that profile, the box settles within a few thousand steps."""
    lat = O.RefLattice(L, L, 1.0, eta, west=(O.VELOCITY, 0, 0), east=(O.VELOCITY, 0, 0),
                       south=(O.VELOCITY, 0, 0), north=(O.VELOCITY, 0, 0), gy=-g, si_rule=rule)
    xc, yc = L / 2 - 0.3, L / 2 + 0.2
    lat.set_disk(xc, yc, r)
    xy, n, ds = W.disk_si_points(xc, yc, r, npts)
    lat.set_si_points(xy, n, ds)
    y = np.arange(L)[:, None] * np.ones((1, L))
    lat.set_fields(1.0 - 3.0 * g * (y - yc), 0.0 * y, 0.0 * y)
    lat.step(steps)
    assert np.abs(lat.ux).max() <= 1e-9 and np.abs(lat.uy).max() <= 1e-9  # at rest
    return lat, (xc, yc, r), (xy, n, ds), g


def test_hydrostatic_archimedes_stress_integration_interpolated():
    # Rule 1 samples sigma at p_i = x_i + 1.5 n_i, bilinear -- exact for the
    # linear pressure.  With rho = rho_c - 3 g (y - y_c):
    #   F = -sum_i S_i (rho(p_i) - rho0)/3 n_i = g sum_i S_i (p_iy - y_c) n_i
    # (the constant part cancels: sum S_i n_i = 0), and for N equally spaced
    # points on the circle, sum S (y - y_c) n_y = pi r^2 and
    # sum S n_y^2 = pi r: F_y = g pi r (r + 1.5), the Archimedes force on the
    # disk grown by the 1.5-cell sampling offset; F_x = 0, and no torque
    # about the centre (the pressure acts along the radius).
    lat, (xc, yc, r), _, g = hydrostatic_box(1)
    assert (lat.si_node4.reshape(-1, 4) >= 0).all()  # every point interpolates
    si = lat.si()[-1]
    fy = g * math.pi * r * (r + 1.5)
    assert abs(si[1] - fy) <= 1e-6 * fy
    assert abs(si[0]) <= 1e-6 * fy and abs(si[2]) <= 1e-6 * fy * r


def test_hydrostatic_archimedes_stress_integration_nearest_node():
    # Rule 0 takes sigma at the sample node r_i itself:
    #   F = g sum_i S_i (y(r_i) - y_c) n_i   (both components)
    lat, (xc, yc, r), (xy, n, ds), g = hydrostatic_box(0)
    node = lat.si_node4.reshape(-1, 4)[:, 0]
    ys = (node // lat.nx).astype(float)
    ref = g * np.array([(ds * (ys - yc) * n[:, 0]).sum(), (ds * (ys - yc) * n[:, 1]).sum()])
    si = lat.si()[-1]
    assert ref[1] > g * math.pi * r * r  # the samples lie outside the disk
    assert np.abs(si[:2] - ref).max() <= 1e-6 * ref[1]


def test_hydrostatic_momentum_exchange_balances_the_body_force():
    # At rest the solid cells' momentum is steady: what streaming brings into
    # them each step (the ME force, Eq. MMEL summed) cancels what their
    # collision adds, the force density G in every solid cell (penalization
    # is idle at u = u_s = 0): F_ME = -G N_solid = (0, g N_solid).
    lat, _, _, g = hydrostatic_box(0)
    nsolid = int((lat.solid != 0).sum())
    me = lat.me()[-1]
    assert abs(me[1] - g * nsolid) <= 1e-6 * g * nsolid
    assert abs(me[0]) <= 1e-6 * g * nsolid


# ----------------------------------------------------------------------------
# stress-integration points of a rotating body (Eqs. dep1, theta2)
# ----------------------------------------------------------------------------

def asymmetric_points(xc, yc, r, npts, seed):
    # points on the circle at random angles, so that no rotation maps the set
    # onto itself with other indices
    th = np.sort(np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi, npts))
    n = np.stack([np.cos(th), np.sin(th)], 1)
    return np.stack([xc + r * n[:, 0], yc + r * n[:, 1]], 1), n, np.full(npts, 2 * math.pi * r / npts)


@pytest.mark.parametrize("theta0", [0.0, 0.3])
def test_rotating_points_quarter_turn(theta0):
    # prescribed rotation by pi/2 in N steps, plus a translation: every
    # registered point and normal (given in the world frame at the body's
    # current angle theta0) is carried rigidly,
    #   x_i -> x_G(N) + R(pi/2) (x_i - x_G(0)),  n_i -> R(pi/2) n_i,
    # R(pi/2) (a, b) = (-b, a): counter-clockwise for omega > 0, the sense of
    # the body's velocity field u_G + omega e_z x (x - x_G)
    xc, yc, r, N = 30.25, 28.5, 6.3, 40
    u, v = 0.011, -0.007
    lat = O.RefLattice(64, 60, 0.8, 1e-3)
    lat.set_disk(xc, yc, r)
    xy, n, ds = asymmetric_points(xc, yc, r, 48, seed=5)
    lat.set_motion(xc, yc, theta0, 0.0, 0.0, 0.0)
    lat.set_si_points(xy, n, ds)
    lat.set_motion(xc, yc, theta0, u, v, (math.pi / 2) / N)
    lat.init_uniform(1.0, 0.0, 0.0)
    lat.step(N)
    assert abs(lat.body.theta - theta0 - math.pi / 2) <= 1e-14
    gx, gy = xc + N * u, yc + N * v
    assert abs(lat.body.x - gx) <= 1e-12 and abs(lat.body.y - gy) <= 1e-12
    want = np.stack([gx - (xy[:, 1] - yc), gy + (xy[:, 0] - xc)], 1)
    assert np.abs(lat.si_xy - want).max() <= 1e-12
    assert np.abs(lat.si_n - np.stack([-n[:, 1], n[:, 0]], 1)).max() <= 1e-14
    assert np.abs(lat.si_ds - ds).max() == 0.0


def test_rotating_points_move_with_the_body_velocity():
    # one step of a spinning, translating body moves each point by the rigid
    # velocity at the point, u_G + omega e_z x (x_i - x_G), up to the
    # second-order term of the rotation (|omega|^2 r / 2)
    xc, yc, r = 30.0, 28.0, 6.0
    u, v, w = 0.02, 0.013, 0.004
    lat = O.RefLattice(64, 60, 0.8, 1e-3)
    lat.set_disk(xc, yc, r)
    xy, n, ds = asymmetric_points(xc, yc, r, 40, seed=9)
    lat.set_si_points(xy, n, ds)
    lat.set_motion(xc, yc, 0.0, u, v, w)
    lat.init_uniform(1.0, 0.0, 0.0)
    lat.step(1)
    vel = np.stack([u - w * (xy[:, 1] - yc), v + w * (xy[:, 0] - xc)], 1)
    err = np.abs(lat.si_xy - xy - vel).max()
    assert err <= 0.5 * w * w * r * (1 + 1e-9)
    assert err >= 0.1 * w * w * r  # the rotation really is of order omega^2 off the chord
