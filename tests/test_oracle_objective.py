"""Pins for the oracle's objective, the integrated wall pressure (no GPU).

J = sum over slip-wall faces of p_w |S|, with the wall pressure of the wall-flux
override of Sec. 7.2 (V7), p_w = 1.5 p_0 - 0.5 p_1 (p_0 the cell next to the
wall, p_1 the next one in).  The values below come from geometry and from the
exactness of that extrapolation on linear data, not from the oracle's own
formula:
  * a uniform state on the compression-ramp grid: J = p (flat length 0.5 +
    ramp length 1 / cos 10 deg) when the corner is a grid node;
  * a pressure linear in x and y on a Cartesian channel with uniform spacing:
    1.5 p_0 - 0.5 p_1 is the exact wall value, and the midpoint sum of a
    linear function is its exact integral, so J = the analytic integral of p
    over both walls;
  * the same on a 3D Cartesian box with slip walls on the k faces.
A planted mistake (p_0 in place of the extrapolation, a wrong face, an area
component in place of |S|) fails at least one of them."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import Problem, gas
import oracle.solver as osolver

P_INF = 1.0 / synth.GAMMA


def _uniform_ramp(ni, nj):
    c = synth.compression_ramp(ni, nj)
    return c


@pytest.mark.parametrize("ni,nj", [(48, 16), (96, 8)])
def test_uniform_state_on_ramp_gives_wall_length(ni, nj):
    # x_i = 1.5 i / ni puts the corner x = 0.5 on node ni / 3
    assert ni % 3 == 0
    c = _uniform_ramp(ni, nj)
    P = Problem(c)
    J = P.wall_pressure_integral(P.initial_state()).item()
    exact = P_INF * (0.5 + 1.0 / math.cos(math.radians(10.0)))
    assert abs(J - exact) <= 1e-13 * exact, (J, exact)


def test_uniform_state_corner_inside_a_face():
    # corner between nodes: the face across it is the straight chord
    ni, nj = 50, 6
    c = _uniform_ramp(ni, nj)
    P = Problem(c)
    J = P.wall_pressure_integral(P.initial_state()).item()
    x = 1.5 * np.arange(ni + 1) / ni
    yw = np.where(x <= 0.5, 0.0, (x - 0.5) * math.tan(math.radians(10.0)))
    length = float(np.sqrt(np.diff(x) ** 2 + np.diff(yw) ** 2).sum())
    assert abs(J - P_INF * length) <= 1e-13 * length
    # and the chord is shorter than the polyline
    assert P_INF * length < P_INF * (0.5 + 1.0 / math.cos(math.radians(10.0)))


def _channel_2d(ni, nj, lx, ly, a, b, cy):
    """Cartesian channel [0, lx] x [0, ly], slip walls at jmin and jmax,
    periodic in i; p = a + b x + cy y at the cell centres."""
    nodes = synth.cartesian_nodes_2d(ni, nj, lx=lx, ly=ly)
    blk = synth.Block(ni, nj, 1, nodes)
    bcs = [synth.full_face_patch(2, blk, 0, synth.JMIN, synth.SLIP_WALL),
           synth.full_face_patch(2, blk, 0, synth.JMAX, synth.SLIP_WALL)]
    conns = [synth.Connection(0, synth.IMIN, [0], [nj], 0, synth.IMAX, [0], [nj], 0)]
    xc = (np.arange(ni) + 0.5) * lx / ni
    yc = (np.arange(nj) + 0.5) * ly / nj
    X, Y = np.meshgrid(xc, yc, indexing="xy")
    prim = np.zeros((4, nj, ni))
    prim[0] = 1.0
    prim[1] = 0.3
    prim[3] = a + b * X + cy * Y
    return synth.Case("channel_2d", 2, [blk], bcs, conns, [prim], synth.Scheme(), 1)


def test_linear_pressure_channel_2d():
    lx, ly, a, b, cy = 1.7, 0.6, 0.8, 0.25, -0.4
    c = _channel_2d(34, 10, lx, ly, a, b, cy)
    P = Problem(c)
    J = P.wall_pressure_integral(P.initial_state()).item()
    # bottom wall: int_0^lx (a + b x) dx; top wall: int_0^lx (a + b x + cy ly) dx
    exact = 2.0 * (a * lx + 0.5 * b * lx * lx) + cy * ly * lx
    assert abs(J - exact) <= 1e-13 * abs(exact), (J, exact)


def test_single_wall_picks_its_own_face():
    # only the top wall: the pressure there is a + b x + cy ly
    lx, ly, a, b, cy = 1.0, 0.5, 0.9, 0.1, 0.7
    c = _channel_2d(20, 8, lx, ly, a, b, cy)
    c.bcs = [c.bcs[1]]
    P = Problem(c)
    J = P.wall_pressure_integral(P.initial_state()).item()
    exact = a * lx + 0.5 * b * lx * lx + cy * ly * lx
    assert abs(J - exact) <= 1e-13 * abs(exact), (J, exact)


def _box_3d(n, lens, coef):
    """Cartesian box, slip walls on kmin and kmax, periodic in i and j;
    p = c0 + c1 x + c2 y + c3 z at the cell centres."""
    ni, nj, nk = n
    lx, ly, lz = lens
    x = np.arange(ni + 1) * lx / ni
    y = np.arange(nj + 1) * ly / nj
    z = np.arange(nk + 1) * lz / nk
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    nodes = np.stack([X, Y, Z]).astype(np.float64)
    blk = synth.Block(ni, nj, nk, nodes)
    bcs = [synth.full_face_patch(3, blk, 0, synth.KMIN, synth.SLIP_WALL),
           synth.full_face_patch(3, blk, 0, synth.KMAX, synth.SLIP_WALL)]
    conns = [cn for cn in synth.periodic_self_connections(3, ni, nj, nk) if cn.face_a in (synth.IMIN, synth.JMIN)]
    xc = (np.arange(ni) + 0.5) * lx / ni
    yc = (np.arange(nj) + 0.5) * ly / nj
    zc = (np.arange(nk) + 0.5) * lz / nk
    Zc, Yc, Xc = np.meshgrid(zc, yc, xc, indexing="ij")
    prim = np.zeros((5, nk, nj, ni))
    prim[0] = 1.0
    prim[1] = 0.2
    c0, c1, c2, c3 = coef
    prim[4] = c0 + c1 * Xc + c2 * Yc + c3 * Zc
    return synth.Case("box_3d", 3, [blk], bcs, conns, [prim], synth.Scheme(), 1)


def test_linear_pressure_box_3d():
    lens = (1.2, 0.7, 0.5)
    coef = (0.9, 0.3, -0.2, 0.6)
    c = _box_3d((6, 5, 4), lens, coef)
    P = Problem(c)
    J = P.wall_pressure_integral(P.initial_state()).item()
    lx, ly, lz = lens
    c0, c1, c2, c3 = coef
    one_wall = lx * ly * (c0 + c1 * lx / 2 + c2 * ly / 2)
    exact = 2.0 * one_wall + c3 * lz * lx * ly
    assert abs(J - exact) <= 1e-13 * abs(exact), (J, exact)


def test_planted_mistakes_fail_a_pin(monkeypatch):
    """The pins above are sensitive to the plausible slips: p_0 for the
    extrapolated wall pressure, and a component of S for |S|."""
    # one wall: with both walls the half-cell errors of p_0 cancel
    lx, ly, a, b, cy = 1.0, 0.5, 0.9, 0.1, 0.7
    case = _channel_2d(20, 8, lx, ly, a, b, cy)
    case.bcs = [case.bcs[1]]
    exact = a * lx + 0.5 * b * lx * lx + cy * ly * lx

    real = osolver.interior_layer

    def first_layer_only(q, dim, face, layer, lo, hi):
        return real(q, dim, face, 0, lo, hi)

    monkeypatch.setattr(osolver, "interior_layer", first_layer_only)
    P = Problem(case)
    J = P.wall_pressure_integral(P.initial_state()).item()
    assert abs(J - exact) > 1e-6 * abs(exact)
    monkeypatch.setattr(osolver, "interior_layer", real)

    # area component in place of |S| on the inclined ramp
    real_slab = osolver.face_area_slab

    def component(S_axis, dim, face, lo, hi):
        s = real_slab(S_axis, dim, face, lo, hi)
        out = torch.zeros_like(s)
        out[1] = s[1]
        return out

    monkeypatch.setattr(osolver, "face_area_slab", component)
    c = _uniform_ramp(48, 8)
    P = Problem(c)
    J = P.wall_pressure_integral(P.initial_state()).item()
    exact = P_INF * (0.5 + 1.0 / math.cos(math.radians(10.0)))
    assert abs(J - exact) > 1e-6 * exact
