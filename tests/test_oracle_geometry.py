"""Pins of the oracle's solid indicator chi (Eq. fcar) and SI sample nodes.

  * disk: brute-force count of lattice points with exact rational arithmetic
    (centre and radius on the 1/4096 grid the mask uses), including the
    Gauss-circle counts for integer centres;
  * polygon: Pick's theorem for lattice polygons (points on the boundary
    count as inside, so the count is A + B/2 + 1), and an exact winding-number
    test with rational arithmetic for random off-grid polygons;
  * NACA 0012: the cell count approaches the closed-form section area;
  * sample nodes: fluid, inside the domain, reached from the nearest node by
    walking away from the body along the direction closest to n.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle as O
import workloads as W

Q = 4096


def q(v):
    return Fr(round(v * Q), Q)


@pytest.mark.parametrize("r", [1, 2, 3, 4, 5, 6, 7, 8, 11])
def test_gauss_circle_counts(r):
    n = 2 * r + 7
    m = O.mask_disk(n, n, r + 3, r + 3, r)
    brute = sum(1 for i in range(-r, r + 1) for j in range(-r, r + 1) if i * i + j * j <= r * r)
    assert int(m.sum()) == brute
    if r == 8:
        assert brute == 197  # the 128x64 channel's disk


def test_disk_off_grid_exact():
    g = np.random.default_rng(7)
    for _ in range(20):
        xc, yc, r = g.uniform(8, 24), g.uniform(8, 24), g.uniform(2, 7)
        m = O.mask_disk(32, 32, xc, yc, r)
        X, Y, R = q(xc), q(yc), q(r)
        for j in range(32):
            for i in range(32):
                assert m[j, i] == int((i - X) ** 2 + (j - Y) ** 2 <= R * R)


def shoelace2(v):
    return sum(v[k][0] * v[(k + 1) % len(v)][1] - v[(k + 1) % len(v)][0] * v[k][1] for k in range(len(v)))


@pytest.mark.parametrize("seed", range(6))
def test_pick_theorem_lattice_polygons(seed):
    # star-shaped lattice polygon around (20, 20)
    g = np.random.default_rng(seed)
    nv = int(g.integers(3, 9))
    ang = np.sort(g.uniform(0, 2 * math.pi, nv))
    rad = g.uniform(4, 15, nv)
    v = [(int(round(20 + r * math.cos(a))), int(round(20 + r * math.sin(a)))) for a, r in zip(ang, rad)]
    v = [p for k, p in enumerate(v) if p != v[k - 1]]
    A2 = shoelace2(v)
    if len(v) < 3 or A2 <= 0:
        pytest.skip("degenerate draw")
    # simple polygon check: star-shaped by construction when angles are distinct
    B = sum(math.gcd(abs(v[(k + 1) % len(v)][0] - v[k][0]), abs(v[(k + 1) % len(v)][1] - v[k][1]))
            for k in range(len(v)))
    m = O.mask_polygon(40, 40, np.array(v, float))
    assert 2 * int(m.sum()) == A2 + B + 2  # I + B = A + B/2 + 1


def winding_inside(px, py, verts):
    """Exact winding number (non-zero rule) with on-boundary = inside."""
    wn = 0
    nv = len(verts)
    for k in range(nv):
        ax, ay = verts[k]
        bx, by = verts[(k + 1) % nv]
        cr = (bx - ax) * (py - ay) - (by - ay) * (px - ax)
        if cr == 0 and min(ax, bx) <= px <= max(ax, bx) and min(ay, by) <= py <= max(ay, by):
            return True
        if ay <= py:
            if by > py and cr > 0:
                wn += 1
        else:
            if by <= py and cr < 0:
                wn -= 1
    return wn != 0


@pytest.mark.parametrize("seed", range(4))
def test_polygon_off_grid_exact(seed):
    g = np.random.default_rng(100 + seed)
    nv = int(g.integers(5, 12))
    ang = np.sort(g.uniform(0, 2 * math.pi, nv))
    rad = g.uniform(3, 9, nv)
    xy = np.stack([12.3 + rad * np.cos(ang), 11.7 + rad * np.sin(ang)], 1)
    m = O.mask_polygon(24, 24, xy)
    verts = [(q(x), q(y)) for x, y in xy]
    for j in range(24):
        for i in range(24):
            assert m[j, i] == int(winding_inside(Fr(i), Fr(j), verts)), (i, j)


def test_polygon_edge_points_inside():
    # axis-aligned rectangle with integer corners: boundary nodes included
    rect = np.array([[2.0, 3.0], [9.0, 3.0], [9.0, 7.0], [2.0, 7.0]])
    m = O.mask_polygon(12, 10, rect)
    assert int(m.sum()) == 8 * 5
    assert m[3, 2] == 1 and m[7, 9] == 1 and m[5, 10] == 0


def test_naca_mask_area():
    case = W.case_naca(chord=200, aoa_deg=10.0)
    m = O.mask_polygon(case.nx, case.ny, case.polygon)
    # closed-form area of the t = 0.12 section: 10 t c^2 (0.2969*2/3 - 0.1260/2
    # - 0.3516/3 + 0.2843/4 - 0.1015/5)
    area = 10 * 0.12 * 200 ** 2 * (0.2969 * 2 / 3 - 0.1260 / 2 - 0.3516 / 3 + 0.2843 / 4 - 0.1015 / 5)
    assert abs(int(m.sum()) - area) <= 0.01 * area
    _, _, ds = W.polygon_si_points(case.polygon)
    assert abs(case.si_n.T @ ds).max() < 1e-12  # closed contour: sum S n = 0


def test_si_sample_nodes_disk():
    nx = ny = 40
    xc, yc, r = 19.6, 20.3, 7.7
    solid = O.mask_disk(nx, ny, xc, yc, r)
    xy, n, ds = W.disk_si_points(xc, yc, r, 128)
    node, missing = O.si_nodes(solid, xy, n)
    assert missing == 0
    for (px, py), (nx_, ny_), k in zip(xy, n, node):
        X, Y = k % nx, k // nx
        assert solid[Y, X] == 0
        r0 = (math.floor(px + 0.5), math.floor(py + 0.5))
        d = (X - r0[0], Y - r0[1])
        if d != (0, 0):
            # walked away from the body, along a direction within 22.5 deg of n
            L = math.hypot(*d)
            assert (d[0] * nx_ + d[1] * ny_) / L >= math.cos(math.radians(22.5)) - 1e-12
            # every node before it on the walk is solid
            step = (int(np.sign(d[0])), int(np.sign(d[1])))
            for j in range(max(abs(d[0]), abs(d[1]))):
                assert solid[r0[1] + j * step[1], r0[0] + j * step[0]] == 1
        # close to the surface
        assert math.hypot(X - xc, Y - yc) - r <= 2.5
