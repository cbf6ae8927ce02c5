"""Pins for the oracle's laminar viscous terms, no GPU.

* Green's-theorem face gradients are exact for linear fields on curvilinear
  2D and 3D grids, boundary faces included (ghost centres and values set from
  the same linear field).
* Viscous residuals of fields whose exact Navier-Stokes viscous terms are
  known in closed form (hand-derived): uniform shear and uniform dilatation
  (constant stresses: momentum terms vanish on any grid; energy = viscous
  heating mu a^2 and 4/3 mu a^2 on Cartesian grids), a parabolic profile
  (d tau_xy/dy = 2 mu), a parabolic temperature (heat conduction 2k).
* Ghost centres across a periodic connection are the neighbour's centres
  moved by the period; pseudo-nodes at block corners average three cells;
  no-slip ghosts negate the velocity; the viscous time-step term.
* Manufactured smooth fields on curvilinear periodic grids: second-order
  convergence of the viscous residual to the continuous viscous terms
  (automatic differentiation of the fields); measured orders 1.98 and 1.90
  for n = 16 -> 32 -> 64.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import Problem, gas, viscous
from oracle.ghosts import fill_ghosts

G = 1.4


def box_case(ni, nj, nk=None, jitter=True, kinds="farfield", mu=0.01, seed=0):
    """Unit square/cube, optionally jittered, all faces of one boundary kind
    (or periodic), uniform state (overwritten by the tests)."""
    dim = 2 if nk is None else 3
    if dim == 2:
        X = synth.jittered_periodic_nodes_2d(ni, nj, seed) if jitter else synth.cartesian_nodes_2d(ni, nj)
        blk = synth.Block(ni, nj, 1, X)
        prim = np.broadcast_to(np.array([1.0, 0.3, 0.1, 1 / G])[:, None, None], (4, nj, ni)).copy()
    else:
        X = synth.jittered_periodic_nodes_3d(ni, nj, nk, seed)
        blk = synth.Block(ni, nj, nk, X)
        prim = np.broadcast_to(np.array([1.0, 0.3, 0.1, 0.05, 1 / G])[:, None, None, None], (5, nk, nj, ni)).copy()
    if kinds == "periodic":
        bcs, conns = [], synth.periodic_self_connections(dim, ni, nj, 1 if nk is None else nk)
    else:
        q = prim[:, (0,) * dim].reshape(-1)
        bcs = [synth.full_face_patch(dim, blk, 0, f, kinds, q if kinds == synth.FARFIELD else None)
               for f in range(2 * dim)]
        conns = []
    sch = synth.Scheme(limiter="vanleer", viscosity=mu)
    return synth.Case("viscous_box", dim, [blk], bcs, conns, [prim], sch, 1)


def linear_setup(case, coef):
    P = Problem(case)
    met = P.metrics()
    X = P.nodes[0].detach()
    padC = viscous.padded_centers(P, [X], [met[0][0]])[0]
    c = torch.tensor(coef, dtype=torch.float64)  # (nval, dim + 1): value = c0 + c . x
    V = c[:, :1, None].reshape(c.shape[0], *([1] * case.dim)) + \
        torch.einsum("vk,k...->v...", c[:, 1:], padC)
    return P, met, X, padC, V


@pytest.mark.parametrize("dims", [(9, 7, None), (6, 5, 4)])
def test_face_gradients_exact_for_linear_fields(dims):
    case = box_case(*dims)
    dim = case.dim
    rng = np.random.default_rng(3)
    coef = rng.normal(size=(3, dim + 1))
    P, met, X, padC, V = linear_setup(case, coef)
    nP = viscous.pseudo_nodes(padC, dim)
    nV = viscous.pseudo_nodes(V, dim)
    for d in range(dim):
        g = viscous.face_gradients(padC, V, nP, nV, dim, d)
        want = torch.tensor(coef[:, 1:]).reshape(3, dim, *([1] * dim))
        assert torch.allclose(g, want.expand_as(g), rtol=0, atol=1e-11), (d, float((g - want).abs().max()))


def test_pseudo_node_corner_averages_three_cells():
    case = box_case(5, 4, jitter=False)
    P = Problem(case)
    padC = viscous.padded_centers(P, [P.nodes[0].detach()], [P.metrics()[0][0]])[0]
    V = torch.arange(float(np.prod(padC.shape[1:])), dtype=torch.float64).reshape(1, *padC.shape[1:])
    nV = viscous.pseudo_nodes(V, 2)
    # node (0, 0): cells (0,0), (-1,0), (0,-1) -> padded (2,2), (2,1), (1,2) as [j, i]
    assert float(nV[0, 0, 0]) == pytest.approx(float(V[0, 2, 2] + V[0, 2, 1] + V[0, 1, 2]) / 3.0)
    # node (2, 1), interior: four cells
    assert float(nV[0, 1, 2]) == pytest.approx(float(V[0, 2:4, 3:5].sum()) / 4.0)
    # mirrored ghost centres of the Cartesian box (h = 1/5 by 1/4): cell (-1, 0)
    # at (-h_x/2, h_y/2), cell (0, nj) at (h_x/2, 1 + h_y/2)
    assert torch.allclose(padC[:, 2, 1], torch.tensor([-0.1, 0.125], dtype=torch.float64), atol=1e-15)
    assert torch.allclose(padC[:, -2, 2], torch.tensor([0.1, 1.125], dtype=torch.float64), atol=1e-15)
    # the pseudo-node position of a Cartesian corner is the mean of the three centres
    nP = viscous.pseudo_nodes(padC, 2)
    assert torch.allclose(nP[:, 0, 0], (padC[:, 2, 2] + padC[:, 2, 1] + padC[:, 1, 2]) / 3.0)


def test_periodic_ghost_centres_are_translated_neighbours():
    case = box_case(8, 6, kinds="periodic")
    P = Problem(case)
    padC = viscous.padded_centers(P, [P.nodes[0].detach()], [P.metrics()[0][0]])[0]
    # ghost column i = -1 is column ni-1 moved by the period (1, 0)
    assert torch.allclose(padC[0, 2:-2, 1], padC[0, 2:-2, -3] - 1.0, atol=1e-14)
    assert torch.allclose(padC[1, 2:-2, 1], padC[1, 2:-2, -3], atol=1e-14)
    assert torch.allclose(padC[1, 1, 2:-2], padC[1, -3, 2:-2] - 1.0, atol=1e-14)


def set_state(case, rho, u, v, p):
    case.prims = [np.stack([rho, u, v, p])]
    return Problem(case)


def cell_xy(n):
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    Y, Xc = np.meshgrid(c, c, indexing="ij")
    return Xc, Y


def viscous_only(P):
    Q = P.initial_state()
    q = [gas.prim_from_cons(x, G) for x in Q]
    met = P.metrics()
    pads = fill_ghosts(P, q, [m[0] for m in met])
    return viscous.viscous_residual(P, pads, P.nodes, met)[0]


def test_uniform_shear_and_dilatation():
    n, mu, a = 16, 0.02, 0.3
    Xc, Y = cell_xy(n)
    one = np.ones_like(Xc)
    # shear u = a y: tau_xy = mu a; energy: d(u tau_xy)/dy = mu a^2
    P = set_state(box_case(n, n, jitter=False, kinds=synth.EXTRAP_OUTFLOW, mu=mu), one, a * Y, 0 * one, one / G)
    Rv = viscous_only(P)[:, 2:-2, 2:-2]
    assert float(Rv[:3].abs().max()) < 1e-13
    assert torch.allclose(Rv[3], torch.full_like(Rv[3], mu * a * a), rtol=1e-12, atol=0)
    # dilatation u = a x: tau_xx = 4/3 mu a, tau_yy = -2/3 mu a; energy 4/3 mu a^2
    P = set_state(box_case(n, n, jitter=False, kinds=synth.EXTRAP_OUTFLOW, mu=mu), one, a * Xc, 0 * one, one / G)
    Rv = viscous_only(P)[:, 2:-2, 2:-2]
    assert float(Rv[:3].abs().max()) < 1e-13
    assert torch.allclose(Rv[3], torch.full_like(Rv[3], 4.0 / 3.0 * mu * a * a), rtol=1e-12, atol=0)


def test_constant_stress_momentum_vanishes_on_curvilinear_grids():
    """A linear velocity field has constant stresses: their flux through the
    closed faces of every cell cancels (momentum Rv = 0) on any grid."""
    for dims in [(10, 8, None), (6, 5, 4)]:
        case = box_case(*dims, kinds=synth.EXTRAP_OUTFLOW)
        dim = case.dim
        P = Problem(case)
        C = viscous.cell_centers(P.nodes[0].detach()).numpy()
        rng = np.random.default_rng(7)
        A = 0.2 * rng.normal(size=(dim, dim))
        vel = [0.3 + sum(A[i, k] * C[k] for k in range(dim)) for i in range(dim)]
        case.prims = [np.stack([np.ones_like(C[0])] + vel + [np.ones_like(C[0]) / G])]
        P = Problem(case)
        Rv = viscous_only(P)
        inner = tuple([slice(None)] + [slice(1, -1)] * dim)
        assert float(Rv[1:-1][inner[:1] + inner[1:]].abs().max()) < 1e-11


def test_parabolic_profiles():
    n, mu = 20, 0.05
    Xc, Y = cell_xy(n)
    one = np.ones_like(Xc)
    # u = y^2: d tau_xy / dy = 2 mu in x-momentum
    P = set_state(box_case(n, n, jitter=False, kinds=synth.EXTRAP_OUTFLOW, mu=mu), one, Y * Y, 0 * one, one / G)
    Rv = viscous_only(P)[:, 2:-2, 2:-2]
    assert torch.allclose(Rv[1], torch.full_like(Rv[1], 2.0 * mu), rtol=1e-10, atol=0)
    assert float(Rv[2].abs().max()) < 1e-12
    # T = gamma p / rho = 1 + x^2 at rest: heat conduction k d2T/dx2 = 2k
    k = mu / ((G - 1.0) * 0.72)
    P = set_state(box_case(n, n, jitter=False, kinds=synth.EXTRAP_OUTFLOW, mu=mu), one, 0 * one, 0 * one,
                  (1.0 + Xc * Xc) / G)
    Rv = viscous_only(P)[:, 2:-2, 2:-2]
    assert float(Rv[:3].abs().max()) < 1e-13
    assert torch.allclose(Rv[3], torch.full_like(Rv[3], 2.0 * k), rtol=1e-10, atol=0)


def test_noslip_ghosts_and_full_residual():
    case = box_case(8, 6, kinds=synth.NOSLIP_WALL)
    P = Problem(case)
    q = [gas.prim_from_cons(x, G) for x in P.initial_state()]
    pad = fill_ghosts(P, q, [m[0] for m in P.metrics()])[0]
    assert torch.equal(pad[1:3, 2:-2, 1], -pad[1:3, 2:-2, 2])
    assert torch.equal(pad[1:3, 2:-2, 0], -pad[1:3, 2:-2, 3])
    assert torch.equal(pad[3, 2:-2, 1], pad[3, 2:-2, 2])
    # the Navier-Stokes residual is the Euler residual minus Rv
    R = P.residual(P.initial_state())[0]
    P.mu = 0.0
    Re = P.residual(P.initial_state())[0]
    P.mu = 0.01
    pads = fill_ghosts(P, q, [m[0] for m in P.metrics()])
    Rv = viscous.viscous_residual(P, pads, P.nodes, P.metrics())[0]
    assert torch.allclose(R, Re - Rv, rtol=0, atol=1e-14)
    assert float(Rv.abs().max()) > 1e-3


def test_viscous_time_step_term():
    """Uniform Cartesian cell h x h at rest (u = 0, c = 1): lambda = 2h
    (acoustic) + 4 max(4/3, gamma/Pr) mu (2 h^2)/h^2."""
    n, mu = 8, 0.03
    h = 1.0 / n
    case = box_case(n, n, jitter=False, kinds=synth.EXTRAP_OUTFLOW, mu=mu)
    one = np.ones((n, n))
    P = set_state(case, one, 0 * one, 0 * one, one / G)
    S, vol = P.metrics()[0]
    dt = P.cell_dt(P.initial_state()[0], S, vol)
    lam = 2.0 * h + 4.0 * max(4.0 / 3.0, G / 0.72) * mu * 2.0
    assert torch.allclose(dt, torch.full_like(dt, h * h / lam), rtol=1e-14)


def _exact_viscous_terms(x, y, fields, mu, k):
    """Continuous viscous terms (d tau_ij / dx_j and d(u_i tau_ij + k dT/dx_j)/dx_j)
    at points (x, y), by automatic differentiation of the given fields."""
    x = x.clone().requires_grad_(True)
    y = y.clone().requires_grad_(True)
    rho, u, v, p = fields(x, y)
    T = G * p / rho

    def d(f, z):
        return torch.autograd.grad(f.sum(), z, create_graph=True)[0]

    ux, uy, vx, vy = d(u, x), d(u, y), d(v, x), d(v, y)
    div = ux + vy
    txx = mu * 2.0 * ux - 2.0 / 3.0 * mu * div
    tyy = mu * 2.0 * vy - 2.0 / 3.0 * mu * div
    txy = mu * (uy + vx)
    thx = u * txx + v * txy + k * d(T, x)
    thy = u * txy + v * tyy + k * d(T, y)
    return torch.stack([d(txx, x) + d(txy, y), d(txy, x) + d(tyy, y), d(thx, x) + d(thy, y)]).detach()


def test_viscous_residual_second_order_on_curvilinear_grids():
    """Manufactured smooth periodic fields on the jittered periodic grid
    family: the discrete viscous residual converges to the continuous viscous
    terms (evaluated by automatic differentiation) at second order."""
    mu = 0.05
    k = mu / ((G - 1.0) * 0.72)
    tp = 2.0 * np.pi

    def fields(x, y):
        rho = 1.0 + 0.1 * torch.sin(tp * x) * torch.sin(tp * y)
        u = 0.3 + 0.1 * torch.cos(tp * x) * torch.sin(tp * y)
        v = 0.1 * torch.sin(tp * (x + y))
        p = (1.0 + 0.1 * torch.cos(tp * (x - y))) / G
        return rho, u, v, p

    errs = []
    for n in (16, 32, 64):
        case = box_case(n, n, kinds="periodic", mu=mu, seed=2)
        P = Problem(case)
        C = viscous.cell_centers(P.nodes[0].detach())
        rho, u, v, p = fields(C[0], C[1])
        case.prims = [torch.stack([rho, u, v, p]).numpy()]
        P = Problem(case)
        Rv = viscous_only(P)
        ex = _exact_viscous_terms(C[0], C[1], fields, mu, k)
        errs.append(float((Rv[1:] - ex).abs().max()))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 1.8, (errs, orders)
