"""Pins of the oracle's full step (streaming, edge rules, penalization,
collision) against flows with closed-form solutions.

  * Poiseuille (body force G, half-way bounce-back walls): the steady profile
    u(y) = G/(2 rho0 nu) (y + 1/2)(ny - 1/2 - y); with BGK and half-way
    bounce-back the parabola is exact at tau = 1/2 + sqrt(3/16) and converges
    at second order otherwise (nu = cs^2 (tau - 1/2), Eq. tauvisco).
  * Couette (moving wall, velocity bounce-back): exact linear profile.
  * Free-slip (symmetry, u.n = 0): a half channel with a specular wall is the
    lower half of a full channel of twice the height.
  * Uniform flow with an inlet, a zero-gradient outlet and free-slip sides is
    an exact fixed point of the scheme.
  * Taylor-Green vortex: kinetic energy decays as exp(-4 nu k^2 t).
  * Penalized walls (solid bands, Eq. 1): first-order convergence to the
    parabola with walls half a cell outside the mask.
  * Mass: the penalization and forcing carry no mass, so sum rho is constant.
  * Convective outflow f(t+1) = (f(t) + U f_inner(t+1)) / (1 + U): uniform
    flow stays a fixed point; U -> infinity is the zero-gradient rule; U = 0
    freezes the incoming populations at their initial values; its steady
    state (f = f_inner) is the zero-gradient one.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W

MAGIC_TAU = 0.5 + math.sqrt(3.0 / 16.0)
G = 1e-6


def channel(ny, tau, north=(O.VELOCITY, 0.0, 0.0), nx=1, steps_factor=20.0, eta=float("inf")):
    nu = (tau - 0.5) / 3.0
    lat = O.RefLattice(nx, ny, tau, eta, south=(O.VELOCITY, 0.0, 0.0), north=north, gx=G)
    lat.init_uniform(1.0, 0.0, 0.0)
    lat.step(int(steps_factor * ny * ny / nu))
    return lat, nu


def test_poiseuille_exact_at_magic_tau():
    ny = 16
    lat, nu = channel(ny, MAGIC_TAU)
    y = np.arange(ny)
    ex = G / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
    assert np.abs(lat.ux[:, 0] - ex).max() <= 1e-9 * ex.max()
    assert np.abs(lat.uy).max() <= 1e-10 * ex.max()


def test_poiseuille_second_order():
    errs = []
    for ny in (8, 16, 32):
        lat, nu = channel(ny, 0.8)
        y = np.arange(ny)
        ex = G / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
        errs.append(np.linalg.norm(lat.ux[:, 0] - ex) / np.linalg.norm(ex))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 1.9, (errs, orders)


def test_couette_linear_profile():
    ny, tau, U = 16, 0.8, 0.01
    nu = (tau - 0.5) / 3
    lat = O.RefLattice(1, ny, tau, float("inf"), south=(O.VELOCITY, 0, 0), north=(O.VELOCITY, U, 0))
    lat.init_uniform(1.0, 0.0, 0.0)
    lat.step(int(30 * ny * ny / nu))
    y = np.arange(ny)
    assert np.abs(lat.ux[:, 0] - U * (y + 0.5) / ny).max() <= 1e-12


def test_couette_moving_wall_in_x_edges():
    # same flow turned by 90 degrees: walls on the west/east edges move in y
    nx, tau, U = 16, 0.8, 0.01
    nu = (tau - 0.5) / 3
    lat = O.RefLattice(nx, 1, tau, float("inf"), west=(O.VELOCITY, 0, 0), east=(O.VELOCITY, 0, U))
    lat.init_uniform(1.0, 0.0, 0.0)
    lat.step(int(30 * nx * nx / nu))
    x = np.arange(nx)
    assert np.abs(lat.uy[0, :] - U * (x + 0.5) / nx).max() <= 1e-12


def test_freeslip_half_channel_south_north():
    ny = 16
    lat, nu = channel(ny, MAGIC_TAU, north=(O.FREESLIP, 0, 0), steps_factor=80.0)
    y = np.arange(ny)
    ex = G / (2 * nu) * (y + 0.5) * (2 * ny - 0.5 - y)
    assert np.abs(lat.ux[:, 0] - ex).max() <= 1e-9 * ex.max()


def test_freeslip_half_channel_west_east():
    nx = 16
    nu = (MAGIC_TAU - 0.5) / 3
    lat = O.RefLattice(nx, 1, MAGIC_TAU, float("inf"), west=(O.FREESLIP, 0, 0), east=(O.VELOCITY, 0, 0), gy=G)
    lat.init_uniform(1.0, 0.0, 0.0)
    lat.step(int(80 * nx * nx / nu))
    x = np.arange(nx)[::-1]  # distance index from the no-slip east wall
    ex = G / (2 * nu) * (x + 0.5) * (2 * nx - 0.5 - x)
    assert np.abs(lat.uy[0, :] - ex).max() <= 1e-9 * ex.max()


@pytest.mark.parametrize("sides", [O.FREESLIP, O.PERIODIC])
def test_uniform_flow_is_a_fixed_point(sides):
    U = 0.05
    lat = O.RefLattice(24, 10, 0.53, float("inf"), west=(O.VELOCITY, U, 0), east=(O.OUTFLOW, 0, 0),
                       south=(sides, 0, 0), north=(sides, 0, 0))
    lat.init_uniform(1.0, U, 0.0)
    f0 = lat.ft.copy()
    lat.step(50)
    assert np.abs(lat.ft - f0).max() <= 1e-14
    assert np.abs(lat.ux - U).max() <= 1e-15


def test_uniform_flow_vertical_outflow_south():
    V = -0.03
    lat = O.RefLattice(8, 20, 0.6, float("inf"), west=(O.FREESLIP, 0, 0), east=(O.FREESLIP, 0, 0),
                       south=(O.OUTFLOW, 0, 0), north=(O.VELOCITY, 0, V))
    lat.init_uniform(1.0, 0.0, V)
    f0 = lat.ft.copy()
    lat.step(40)
    assert np.abs(lat.ft - f0).max() <= 1e-14


def taylor_green(L, tau, U0=0.01, steps=None):
    nu = (tau - 0.5) / 3
    k = 2 * math.pi / L
    x = np.arange(L)[None, :]
    y = np.arange(L)[:, None]
    ux = -U0 * np.cos(k * x) * np.sin(k * y)
    uy = U0 * np.sin(k * x) * np.cos(k * y)
    p = -U0 ** 2 / 4 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    lat = O.RefLattice(L, L, tau, float("inf"))
    lat.set_fields(1.0 + 3.0 * p, ux + 0 * p, uy + 0 * p)
    steps = steps or int(0.5 / (2 * nu * k * k))
    E = []
    for _ in range(steps):
        lat.step(1)
        E.append((lat.rho * (lat.ux ** 2 + lat.uy ** 2)).sum())
    return lat, np.array(E), nu, k, ux, uy


def test_taylor_green_viscosity_and_order():
    rel_nu, errs = [], []
    for L in (32, 64):
        lat, E, nu, k, ux0, uy0 = taylor_green(L, 0.8)
        n = len(E)
        t = np.arange(1, n + 1)
        slope = np.polyfit(t[n // 4:], np.log(E[n // 4:]), 1)[0]
        rel_nu.append(abs(-slope / (4 * k * k) / nu - 1))
        dec = math.exp(-2 * nu * k * k * n)
        errs.append(math.sqrt(((lat.ux - ux0 * dec) ** 2 + (lat.uy - uy0 * dec) ** 2).sum()
                              / ((ux0 * dec) ** 2 + (uy0 * dec) ** 2).sum()))
    assert rel_nu[1] <= 0.01
    assert math.log2(errs[0] / errs[1]) >= 1.9


def test_penalized_walls_first_order():
    errs = []
    eta = 1e-4
    for H in (8, 16, 32):
        tau, band = 0.8, 4
        nu = (tau - 0.5) / 3
        ny = H + 2 * band
        lat = O.RefLattice(1, ny, tau, eta, gx=G)
        m = np.zeros((ny, 1), np.uint8)
        m[:band] = 1
        m[band + H:] = 1
        lat.set_mask(m)
        lat.init_uniform(1.0, 0.0, 0.0)
        lat.step(int(15 * H * H / nu))
        yy = np.arange(ny) - band
        fl = (yy >= 0) & (yy < H)
        ex = G / (2 * nu) * (yy + 0.5) * (H - 0.5 - yy)
        u = lat.ux[:, 0]
        errs.append(np.linalg.norm(u[fl] - ex[fl]) / np.linalg.norm(ex[fl]))
        assert np.abs(u[~fl]).max() <= eta * ex.max()
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 0.9, (errs, orders)


def test_mass_conservation_with_penalized_disk():
    L = 48
    lat = O.RefLattice(L, L, 0.6, 1e-4)
    lat.set_disk(20.3, 23.7, 6.2)
    ux, uy = W.smooth_random_velocity(L, L, seed=11, amp=0.03)
    rho = W.random_density(L, L, seed=12, amp=1e-3)
    lat.set_fields(rho, ux, uy)
    m0 = math.fsum(lat.ft.ravel())
    lat.step(2000)
    m1 = math.fsum(lat.ft.ravel())
    # Exact arithmetic conserves mass exactly, and so does the oracle up to
    # unbiased rounding (a few 1e-16 over 2000 steps): its weights sum to one
    # exactly in binary.  With the nearest doubles of 4/9, 1/9 and 1/36 the
    # sum falls 2^-54 short and the mass would drift by 2000 * 2^-54 / tau =
    # 1.85e-13.  A dropped or misplaced mass term would show up orders of
    # magnitude above the bound, which is 10x tighter than 1e-13.
    assert abs(m1 - m0) / m0 <= 1e-14


# ---------------------------------------------------------------------------
# two-relaxation-time collision (Eq. TRT)
# ---------------------------------------------------------------------------

def trt_channel(ny, tau, lam):
    nu = (tau - 0.5) / 3.0
    lat = O.RefLattice(1, ny, tau, float("inf"), south=(O.VELOCITY, 0, 0), north=(O.VELOCITY, 0, 0), gx=G,
                       trt_lambda=lam)
    lat.init_uniform(1.0, 0.0, 0.0)
    lat.step(int(30 * ny * ny / nu) if tau > 0.6 else 40000)
    y = np.arange(ny)
    return lat.ux[:, 0], G / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)


@pytest.mark.parametrize("tau", [0.55, 1.2])
def test_trt_poiseuille_exact_for_lambda_3_16(tau):
    # with half-way bounce-back, TRT places the wall exactly half a link out
    # for Lambda = 3/16, whatever tau
    u, ex = trt_channel(16, tau, 3.0 / 16.0)
    assert np.abs(u - ex).max() <= 1e-9 * ex.max()


def test_trt_steady_state_depends_on_lambda_only():
    # the paper's Lambda = 1/6: same steady profile (relative to nu) for two taus
    u1, ex1 = trt_channel(12, 0.55, 1.0 / 6.0)
    u2, ex2 = trt_channel(12, 1.2, 1.0 / 6.0)
    assert np.abs(u1 / ex1.max() - u2 / ex2.max()).max() <= 1e-9
    assert np.abs(u1 - ex1).max() > 1e-5 * ex1.max()  # not the exact case


def test_trt_with_equal_rates_is_bgk():
    tau = 0.7
    lam = (tau - 0.5) ** 2  # tau- = tau+
    a = O.RefLattice(40, 30, tau, 1e-4, trt_lambda=lam)
    b = O.RefLattice(40, 30, tau, 1e-4)
    for lat in (a, b):
        lat.set_disk(19.3, 14.8, 6.1)
        ux, uy = W.smooth_random_velocity(40, 30, seed=41, amp=0.03)
        lat.set_fields(W.random_density(40, 30, seed=42), ux, uy)
        lat.step(30)
    assert np.abs(a.ft - b.ft).max() <= 1e-14
    assert np.abs(a.me()[-1] - b.me()[-1]).max() <= 1e-12


# ----------------------------------------------------------------------------
# convective outflow edge
# ----------------------------------------------------------------------------

def disk_channel_lattice(east, south=(O.FREESLIP, 0, 0), north=(O.FREESLIP, 0, 0), tau=0.6, nx=40, ny=18):
    lat = O.RefLattice(nx, ny, tau, 1e-3, west=(O.VELOCITY, 0.04, 0), east=east, south=south, north=north)
    lat.set_disk(14.3, 8.6, 3.7)
    ux, uy = W.smooth_random_velocity(nx, ny, seed=4, amp=0.02)
    lat.set_fields(W.random_density(nx, ny, seed=5, amp=1e-3), 0.04 + ux, uy)
    return lat


@pytest.mark.parametrize("sides", [O.FREESLIP, O.PERIODIC])
def test_convective_uniform_flow_is_a_fixed_point(sides):
    U = 0.05
    lat = O.RefLattice(24, 10, 0.53, float("inf"), west=(O.VELOCITY, U, 0), east=(O.CONVECTIVE, U, 0),
                       south=(sides, 0, 0), north=(sides, 0, 0))
    lat.init_uniform(1.0, U, 0.0)
    f0 = lat.ft.copy()
    lat.step(50)
    assert np.abs(lat.ft - f0).max() <= 1e-14


def test_convective_vertical_uniform_flow_is_a_fixed_point():
    V = -0.03
    lat = O.RefLattice(8, 20, 0.6, float("inf"), west=(O.FREESLIP, 0, 0), east=(O.FREESLIP, 0, 0),
                       south=(O.CONVECTIVE, 0.03, 0), north=(O.VELOCITY, 0, V))
    lat.init_uniform(1.0, 0.0, V)
    f0 = lat.ft.copy()
    lat.step(40)
    assert np.abs(lat.ft - f0).max() <= 1e-14


def test_convective_infinite_speed_is_zero_gradient():
    a = disk_channel_lattice((O.CONVECTIVE, 1e12, 0))
    b = disk_channel_lattice((O.OUTFLOW, 0, 0))
    for _ in range(6):
        a.step(5)
        b.step(5)
        assert np.abs(a.ft - b.ft).max() <= 1e-10


def test_convective_zero_speed_freezes_incoming_populations():
    # U = 0: the populations entering through the east edge keep their initial
    # streamed values exactly, while the flow inside evolves
    lat = disk_channel_lattice((O.CONVECTIVE, 0.0, 0))
    f0 = lat.ft.copy()
    inflow = [3, 6, 7]  # c_x < 0
    for _ in range(4):
        lat.step(7)
        assert np.array_equal(lat.streamed()[:, -1, inflow], f0[:, -1, inflow])
    assert np.abs(lat.ft[:, :-1] - f0[:, :-1]).max() > 1e-6


@pytest.mark.parametrize("U", [0.37, 0.02])
def test_convective_one_step_blend(U):
    # periodic south/north, so the inner value of incoming population a at
    # (nx-1, y) is ft[(y - c_y) mod ny, nx-1, a] (the zero-gradient source).
    # (i) previous value = inner value: the step equals the zero-gradient
    # step; (ii) previous value = inner value + d: the incoming populations
    # come out as the zero-gradient ones + d / (1 + U), nothing else changes
    per = (O.PERIODIC, 0, 0)
    a = disk_channel_lattice((O.CONVECTIVE, U, 0), south=per, north=per)
    b = disk_channel_lattice((O.OUTFLOW, 0, 0), south=per, north=per)
    a.step(9)
    b.ft[:] = a.ft
    ny = a.ny
    inner = np.zeros((ny, 9))
    for k in (3, 6, 7):
        inner[:, k] = a.ft[(np.arange(ny) - O.CY[k]) % ny, -1, k]
    d = np.zeros((ny, 9))
    d[:, [3, 6, 7]] = np.random.default_rng(1).normal(0.0, 1e-3, (ny, 3))
    for dd in (0.0 * d, d):
        a.ft[:] = b.ft
        a.fprev[:, -1, :] = inner + dd
        a.step(1)
        b2 = disk_channel_lattice((O.OUTFLOW, 0, 0), south=per, north=per)
        b2.ft[:] = b.ft
        b2.step(1)
        s_a, s_b = a.streamed(), b2.streamed()
        expect = s_b.copy()
        expect[:, -1, :] += dd / (1.0 + U)
        assert np.abs(s_a - expect).max() <= 2e-16
