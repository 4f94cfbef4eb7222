"""Pins of the oracle's per-cell algebra against closed forms.

Each check is a moment identity or closed form that the mathematics fixes,
not a retyping of the oracle's own formula:
  * f^eq (Sec. 2.2): zeroth, first and second moments of the D2Q9 equilibrium;
  * forcing term (Guo et al. 2002, cited for F_alpha): moments 0 / F / uF + Fu;
  * penalized velocity (Eq. updatestepm): the relaxation of u towards u_s in
    a solid cell, |u - u_s| = |m/rho - u_s| / (1 + 1/(2 eta));
  * collision: mass conserved, post-collision momentum = m + F (the
    half-force shift of Eq. updatestep makes the forcing exact).
"""
import ctypes as C
import math

from fractions import Fraction

import numpy as np
import pytest

import oracle as O

CX, CY = O.CX, O.CY


def rng_cells(n, seed):
    g = np.random.default_rng(seed)
    rho = 1.0 + 0.05 * g.standard_normal(n)
    ux = 0.08 * g.standard_normal(n)
    uy = 0.08 * g.standard_normal(n)
    return rho, ux, uy


def test_weights_and_velocity_set():
    # sum w = 1, isotropy sum w c c = cs^2 I, sum w c_x^2 c_y^2 = cs^4
    assert abs(O.W.sum() - 1.0) < 1e-15
    # the stored weights sum to one exactly (rational arithmetic on the
    # doubles), so f^eq carries exactly rho: the zeroth moment that defines it
    assert sum(Fraction(float(w)) for w in O.W) == 1
    for k, ref in ((0, Fraction(4, 9)), (1, Fraction(1, 9)), (5, Fraction(1, 36))):
        assert abs(Fraction(float(O.W[k])) - ref) <= Fraction(1, 2 ** 53) * ref
    f = O.equilibrium(1.0, 0.0, 0.0)  # the oracle's own weights
    assert sum(Fraction(float(v)) for v in f) == 1
    assert abs((O.W * CX * CX).sum() - 1 / 3) < 1e-15
    assert abs((O.W * CX * CY).sum()) < 1e-15
    assert abs((O.W * CX ** 2 * CY ** 2).sum() - 1 / 9) < 1e-15


def test_equilibrium_moments():
    rho, ux, uy = rng_cells(64, 1)
    for r, a, b in zip(rho, ux, uy):
        f = O.equilibrium(r, a, b)
        assert abs(f.sum() - r) <= 1e-15 * r
        assert abs((CX * f).sum() - r * a) <= 2e-16
        assert abs((CY * f).sum() - r * b) <= 2e-16
        # second moment: rho cs^2 I + rho u u
        assert abs((CX * CX * f).sum() - (r / 3 + r * a * a)) <= 2e-15
        assert abs((CX * CY * f).sum() - r * a * b) <= 2e-16
        assert abs((CY * CY * f).sum() - (r / 3 + r * b * b)) <= 2e-15


def test_equilibrium_rest_state_is_weights():
    f = O.equilibrium(1.0, 0.0, 0.0)
    assert np.array_equal(f, O.W * 1.0)


def test_forcing_moments():
    rho, ux, uy = rng_cells(64, 2)
    g = np.random.default_rng(3)
    for a, b in zip(ux, uy):
        Fx, Fy = 1e-3 * g.standard_normal(2)
        s = O.forcing(a, b, Fx, Fy)
        assert abs(s.sum()) < 1e-18
        assert abs((CX * s).sum() - Fx) < 1e-18
        assert abs((CY * s).sum() - Fy) < 1e-18
        assert abs((CX * CX * s).sum() - 2 * a * Fx) < 1e-18
        assert abs((CX * CY * s).sum() - (a * Fy + b * Fx)) < 1e-18
        assert abs((CY * CY * s).sum() - 2 * b * Fy) < 1e-18


def _macro(lat, f, chi, usx, usy):
    out = [C.c_double() for _ in range(5)]
    O.lib().orc_cell_macro(C.byref(lat.p), np.ascontiguousarray(f), chi, usx, usy, *[C.byref(o) for o in out])
    return [o.value for o in out]


@pytest.mark.parametrize("eta", [1e-2, 1e-4, 1e-6])
def test_penalized_velocity_closed_form(eta):
    # In a solid cell without external force, Eq. updatestepm gives
    # u - u_s = (m/rho - u_s) / (1 + 1/(2 eta)).
    lat = O.RefLattice(1, 1, 0.7, eta)
    g = np.random.default_rng(4)
    for _ in range(32):
        f = O.equilibrium(1.0 + 0.02 * g.standard_normal(), *(0.05 * g.standard_normal(2)))
        f = f + 1e-3 * g.standard_normal(9)
        usx, usy = 0.03 * g.standard_normal(2)
        rho, ux, uy, Fx, Fy = _macro(lat, f, 1, usx, usy)
        mx, my = (CX * f).sum(), (CY * f).sum()
        k = 1.0 / (1.0 + 1.0 / (2 * eta))
        assert abs((ux - usx) - (mx / rho - usx) * k) <= 1e-13 * abs(mx / rho - usx) + 1e-18
        assert abs((uy - usy) - (my / rho - usy) * k) <= 1e-13 * abs(my / rho - usy) + 1e-18
        # the force density equals -rho/eta (u - u_s) (penalization term of Eq. 1)
        assert abs(Fx + rho / eta * (ux - usx)) <= 1e-9 * max(abs(Fx), 1e-12)
        assert abs(Fy + rho / eta * (uy - usy)) <= 1e-9 * max(abs(Fy), 1e-12)
        # half-force shift of Eq. updatestep: rho u = m + F/2
        assert abs(rho * ux - (mx + 0.5 * Fx)) <= 1e-15
        assert abs(rho * uy - (my + 0.5 * Fy)) <= 1e-15


def test_fluid_cell_is_plain_lbm():
    lat = O.RefLattice(1, 1, 0.7, 1e-4, gx=2e-5, gy=-1e-5)
    f = O.equilibrium(1.01, 0.03, -0.02) + 1e-4
    rho, ux, uy, Fx, Fy = _macro(lat, f, 0, 0.5, 0.5)
    assert abs(rho - f.sum()) < 1e-15
    assert abs(ux - ((CX * f).sum() + 1e-5) / rho) < 1e-16
    assert abs(uy - ((CY * f).sum() - 0.5e-5) / rho) < 1e-16
    assert (Fx, Fy) == (2e-5, -1e-5)


@pytest.mark.parametrize("chi", [0, 1])
def test_collision_conserves_mass_and_applies_force(chi):
    # A 1x1 fully periodic lattice streams every population onto itself, so
    # one oracle step is exactly one collision of one cell.
    g = np.random.default_rng(5 + chi)
    lat = O.RefLattice(1, 1, 0.63, 1e-3, gx=3e-6, gy=-2e-6)
    if chi:
        lat.set_mask(np.ones((1, 1), np.uint8))
        lat.body.u, lat.body.v = 0.01, -0.02
    for _ in range(16):
        f0 = O.equilibrium(1.0 + 0.02 * g.standard_normal(), *(0.05 * g.standard_normal(2)))
        f0 = f0 + 2e-3 * g.standard_normal(9)
        lat.ft[0, 0, :] = f0
        lat.step(1)
        f1 = lat.ft[0, 0, :]
        rho, ux, uy, Fx, Fy = _macro(lat, f0, chi, 0.01 if chi else 0.0, -0.02 if chi else 0.0)
        assert abs(f1.sum() - f0.sum()) <= 2e-15
        assert abs((CX * f1).sum() - ((CX * f0).sum() + Fx)) <= 1e-15
        assert abs((CY * f1).sum() - ((CY * f0).sum() + Fy)) <= 1e-15
        # non-conserved moments relax with 1/tau towards equilibrium:
        # (Pi~ - Pi_eq) = (1 - 1/tau)(Pi - Pi_eq) + (1 - 1/(2 tau)) Pi_F
        feq = O.equilibrium(rho, ux, uy)
        s = O.forcing(ux, uy, Fx, Fy)
        for mom in (CX * CY, CX * CX - CY * CY):
            lhs = (mom * (f1 - feq)).sum()
            rhs = (1 - 1 / 0.63) * (mom * (f0 - feq)).sum() + (1 - 1 / 1.26) * (mom * s).sum()
            assert abs(lhs - rhs) <= 1e-15
