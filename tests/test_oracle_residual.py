"""Pins for the oracle's residual, ghost fill, time step and Runge-Kutta update (no GPU)."""
import copy
import json
import math
import os

import numpy as np
import pytest
import torch

import synth
from oracle import Problem, gas, metrics

HERE = os.path.dirname(os.path.abspath(__file__))


def residual(case):
    P = Problem(case)
    return P, P.residual(P.initial_state())


def uniform(case, prim):
    c = copy.deepcopy(case)
    for b, q in enumerate(c.prims):
        c.prims[b] = np.broadcast_to(np.asarray(prim, float)[:, None, None] if q.ndim == 3
                                     else np.asarray(prim, float)[:, None, None, None], q.shape).copy()
    return c


# -- freestream preservation -------------------------------------------------

@pytest.mark.parametrize("lim", ["vanleer", "vanalbada", "none"])
def test_freestream_jittered_2d(lim):
    c = uniform(synth.jittered_periodic_square(24, 20, seed=1, limiter=lim), [1.0, 0.7, -0.3, 1 / 1.4])
    _, R = residual(c)
    assert R[0].abs().max() < 1e-12


def test_freestream_jittered_3d():
    c = uniform(synth.jittered_periodic_box(dims=(10, 9, 8), seed=2), [1.0, 0.8, 0.2, -0.1, 1 / 1.4])
    _, R = residual(c)
    assert R[0].abs().max() < 1e-12


def test_freestream_ramp_all_inflow():
    c = synth.compression_ramp(36, 24)
    for p in c.bcs:
        p.kind, p.params = synth.SUP_INFLOW, c.meta["inflow"]
    _, R = residual(c)
    assert R[0].abs().max() < 1e-11


def test_flat_wall_preserves_parallel_flow():
    # ramp grid before the corner is a flat wall; use a straight channel
    c = synth.compression_ramp(30, 16)
    c.blocks[0].nodes = synth.cartesian_nodes_2d(30, 16, lx=1.5)
    _, R = residual(c)
    assert R[0].abs().max() < 1e-12


# -- conservation ------------------------------------------------------------

def test_discrete_conservation_2d():
    c = synth.jittered_periodic_square(24, 20, seed=4)
    P, R = residual(c)
    vol = P.metrics()[0][1]
    tot = (R[0] * vol).sum(dim=(1, 2))
    assert tot.abs().max() < 1e-14


def test_discrete_conservation_3d_and_over_steps():
    c = synth.jittered_periodic_box(dims=(8, 8, 6), seed=5)
    P = Problem(c)
    Q = P.initial_state()
    vol = P.metrics()[0][1]
    R = P.residual(Q)
    assert (R[0] * vol).sum(dim=(1, 2, 3)).abs().max() < 1e-14
    m0 = (Q[0] * vol).sum(dim=(1, 2, 3))
    Q, _ = P.run(Q, 5)
    m1 = (Q[0] * vol).sum(dim=(1, 2, 3))
    assert (m1 - m0).abs().max() < 1e-13


# -- symmetries / topology ---------------------------------------------------

def test_transpose_symmetry_2d():
    c = synth.jittered_periodic_square(16, 12, seed=6)
    P, R = residual(c)
    t = copy.deepcopy(c)
    X = c.blocks[0].nodes
    t.blocks[0] = synth.Block(12, 16, 1, np.stack([X[1].T, X[0].T]).copy())
    q = c.prims[0]
    t.prims[0] = np.stack([q[0].T, q[2].T, q[1].T, q[3].T]).copy()
    t.conns = synth.periodic_self_connections(2, 12, 16)
    _, Rt = residual(t)
    Rt = Rt[0]
    back = torch.stack([Rt[0].T, Rt[2].T, Rt[1].T, Rt[3].T])
    assert torch.allclose(back, R[0], rtol=0, atol=1e-12 * R[0].abs().max())


@pytest.mark.parametrize("base", ["periodic", "ramp"])
def test_block_split_invariance_2d(base):
    if base == "periodic":
        c = synth.jittered_periodic_square(24, 18, seed=7)
    else:
        c = synth.compression_ramp(30, 18)
        c.prims[0] = c.prims[0] * (1 + 0.05 * np.random.default_rng(1).standard_normal(c.prims[0].shape))
    _, R = residual(c)
    s = synth.split_block_case(c, [7, 16], [5, 11])
    _, Rs = residual(s)
    ib, jb = [0, 7, 16, c.blocks[0].ni], [0, 5, 11, c.blocks[0].nj]
    for b in range(3):
        for a in range(3):
            sub = R[0][:, jb[b]:jb[b + 1], ib[a]:ib[a + 1]]
            assert torch.allclose(Rs[b * 3 + a], sub, rtol=0, atol=1e-13 * R[0].abs().max())


def test_reversed_connection_2d():
    """Block B rotated by 180 degrees (both indices reversed) and joined
    imax-to-imax with orient = 1 gives the same residual as the plain split."""
    c = synth.jittered_periodic_square(20, 14, seed=8)
    _, R = residual(c)
    s = synth.split_block_case(c, [9], [])
    A, B = s.blocks
    Bn = synth.Block(B.ni, B.nj, 1, B.nodes[:, ::-1, ::-1].copy())
    qB = s.prims[1][:, ::-1, ::-1].copy()
    nj = A.nj
    conns = [synth.Connection(0, synth.IMAX, [0], [nj], 1, synth.IMAX, [0], [nj], 1),
             synth.Connection(0, synth.IMIN, [0], [nj], 1, synth.IMIN, [0], [nj], 1),
             synth.Connection(0, synth.JMIN, [0], [A.ni], 0, synth.JMAX, [0], [A.ni], 0),
             synth.Connection(1, synth.JMIN, [0], [B.ni], 1, synth.JMAX, [0], [B.ni], 0)]
    r = synth.Case("rev", 2, [A, Bn], [], conns, [s.prims[0], qB], c.scheme, 1)
    _, Rr = residual(r)
    scale = R[0].abs().max()
    assert torch.allclose(Rr[0], R[0][:, :, :9], rtol=0, atol=1e-13 * scale)
    assert torch.allclose(Rr[1].flip(1, 2), R[0][:, :, 9:], rtol=0, atol=1e-13 * scale)


def test_swapped_connection_3d():
    """Second block rotated about the i axis (j' = k, k' = nj-1-j) and joined
    with orient = 6 (swap + reverse second) gives the unsplit residual."""
    ni, nj, nk, cut = 10, 6, 6, 4
    c = synth.jittered_periodic_box(dims=(ni, nj, nk), seed=9)
    _, R = residual(c)
    X, q = c.blocks[0].nodes, c.prims[0]
    XA, qA = X[:, :, :, :cut + 1].copy(), q[:, :, :, :cut].copy()
    XB, qB = X[:, :, :, cut:], q[:, :, :, cut:]
    # rotated B: new axes (k', j', i) with j' = k and k' = nj - 1 - j  -> tensor index [j_rev, k, i]
    XBr = XB.transpose(0, 2, 1, 3)[:, ::-1].copy()
    qBr = qB.transpose(0, 2, 1, 3)[:, ::-1].copy()
    nB = ni - cut
    A = synth.Block(cut, nj, nk, XA)
    B = synth.Block(nB, nk, nj, XBr)
    conns = [synth.Connection(0, synth.IMAX, [0, 0], [nj, nk], 1, synth.IMIN, [0, 0], [nk, nj], 6),
             synth.Connection(1, synth.IMAX, [0, 0], [nk, nj], 0, synth.IMIN, [0, 0], [nj, nk], 5),
             synth.Connection(0, synth.JMIN, [0, 0], [cut, nk], 0, synth.JMAX, [0, 0], [cut, nk], 0),
             synth.Connection(0, synth.KMIN, [0, 0], [cut, nj], 0, synth.KMAX, [0, 0], [cut, nj], 0),
             synth.Connection(1, synth.JMIN, [0, 0], [nB, nj], 1, synth.JMAX, [0, 0], [nB, nj], 0),
             synth.Connection(1, synth.KMIN, [0, 0], [nB, nk], 1, synth.KMAX, [0, 0], [nB, nk], 0)]
    r = synth.Case("rot", 3, [A, B], [], conns, [qA, qBr], c.scheme, 1)
    _, Rr = residual(r)
    scale = R[0].abs().max()
    assert torch.allclose(Rr[0], R[0][..., :cut], rtol=0, atol=1e-13 * scale)
    back = Rr[1].flip(1).transpose(1, 2)
    assert torch.allclose(back, R[0][..., cut:], rtol=0, atol=1e-13 * scale)


# -- time step and Runge-Kutta ----------------------------------------------

def test_cartesian_time_step_closed_form():
    c = uniform(synth.gaussian_bump_periodic(64, 64), [1.0, 0.5, 0.0, 1 / 1.4])
    P = Problem(c)
    dt = P.time_step(P.initial_state())
    assert dt.item() == pytest.approx(0.5 * (1 / 64) / (0.5 + 2.0), rel=1e-14)


@pytest.mark.parametrize("stages", [2, 4])
def test_rk_amplification_polynomial(stages):
    c = synth.gaussian_bump_periodic(8, 8)
    c.scheme.rk_stages = stages
    P = Problem(c)
    lam, dt = 0.7, 0.9
    Q0 = P.initial_state()
    Q1, _ = P.rk_step(Q0, dt=torch.tensor(dt), residual_fn=lambda Qs: [lam * Q for Q in Qs])
    z = -lam * dt
    poly = sum(z ** m / math.factorial(m) for m in range(stages + 1))
    assert torch.allclose(Q1[0], poly * Q0[0], rtol=1e-14)


def test_classic4_amplification_polynomial():
    """Classical RK4 on the linear residual R = lam Q: one step multiplies Q by
    the degree-4 Taylor polynomial of exp(-lam dt)."""
    c = synth.gaussian_bump_periodic(8, 8)
    c.scheme.rk_scheme = "classic4"
    P = Problem(c)
    lam, dt = 0.7, 0.9
    Q0 = P.initial_state()
    Q1, _ = P.rk_step(Q0, dt=torch.tensor(dt), residual_fn=lambda Qs: [lam * Q for Q in Qs])
    z = -lam * dt
    poly = sum(z ** m / math.factorial(m) for m in range(5))
    assert torch.allclose(Q1[0], poly * Q0[0], rtol=1e-14)


@pytest.mark.parametrize("scheme,order", [("classic4", 4), ("mstage", 2)])
def test_rk_order_on_a_nonlinear_ode(scheme, order):
    """dQ/dt = -Q^2 from Q = 1 to t = 1 (exact 1/2) with the residual
    R(Q) = Q^2: halving dt divides the error by 2^order -- four for the
    classical method, two for the four-stage scheme of Sec. 2 (fourth order
    only for linear problems).  A wrong weight or node in either scheme
    changes the ratio."""
    c = synth.gaussian_bump_periodic(4, 4)
    c.scheme.rk_scheme = scheme
    P = Problem(c)
    errs = []
    for n in (20, 40, 80):
        Q = [torch.ones_like(q) for q in P.initial_state()]
        for _ in range(n):
            Q, _ = P.rk_step(Q, dt=torch.tensor(1.0 / n), residual_fn=lambda Qs: [q * q for q in Qs])
        errs.append(float((Q[0] - 0.5).abs().max()))
    for a, b in zip(errs, errs[1:]):
        assert abs(math.log2(a / b) - order) < 0.1, (scheme, errs)


@pytest.mark.parametrize("lim", ["vanleer", "vanalbada"])
def test_entropy_wave_keeps_p_and_u_uniform(lim):
    c = synth.gaussian_bump_periodic(24, 24, limiter=lim)
    P = Problem(c)
    Q, _ = P.run(P.initial_state(), 30)
    q = gas.prim_from_cons(Q[0], P.gamma)
    assert (q[1] - 0.5).abs().max() < 1e-13
    assert q[2].abs().max() < 1e-13
    assert (q[3] - 1 / 1.4).abs().max() < 1e-13
    assert (q[0] - 1).max() > 1e-3  # the bump is still there


@pytest.mark.slow
def test_entropy_wave_second_order_convergence():
    """rho converges to the translated Gaussian at second order (L1)."""
    errs = []
    T = 0.1
    for n in (32, 64, 128):
        c = synth.gaussian_bump_periodic(n, n, limiter="vanleer")
        c.scheme.dt_fixed = 0.2 / n
        P = Problem(c)
        steps = int(round(T / c.scheme.dt_fixed))
        Q, _ = P.run(P.initial_state(), steps)
        xc = c.meta["bump_centre"] + np.array([0.5 * T, 0.0])
        X, Y = synth.cell_centres_index_space(n, n)
        exact = np.ones_like(X)
        for m in (-1, 0, 1):
            for k in (-1, 0, 1):
                exact += 0.01 * np.exp(-((X - xc[0] - m) ** 2 + (Y - xc[1] - k) ** 2) / 0.02)
        errs.append(np.abs(Q[0][0].numpy() - exact).mean())
    order = math.log2(errs[1] / errs[2])
    assert order > 1.6, errs


# -- method of manufactured solutions ---------------------------------------

def _mapped_nodes(N, extra=0):
    s = (np.arange(-extra, N + extra + 1) / N)
    S, T = np.meshgrid(s, s, indexing="xy")
    x = S + 0.04 * np.sin(2 * np.pi * S) * np.sin(2 * np.pi * T)
    y = T + 0.03 * np.sin(2 * np.pi * S + 0.5) * np.cos(2 * np.pi * T)
    return np.stack([x, y])


def _ms_prims(x, y):
    rho = 1.0 + 0.2 * torch.sin(2 * x + 0.3) * torch.cos(1.5 * y)
    u = 0.6 + 0.1 * torch.cos(1.7 * x) * torch.sin(2.2 * y + 0.1)
    v = -0.2 + 0.15 * torch.sin(1.3 * x + 1.9 * y)
    p = 1 / 1.4 + 0.1 * torch.cos(2.4 * x - 0.4) * torch.cos(1.1 * y + 0.2)
    return torch.stack([rho, u, v, p])


def _exact_divergence(x, y, gamma=1.4):
    x = x.clone().requires_grad_(True)
    y = y.clone().requires_grad_(True)
    q = _ms_prims(x, y)
    rho, u, v, p = q
    E = p / (gamma - 1) + 0.5 * rho * (u * u + v * v)
    Fx = [rho * u, rho * u * u + p, rho * u * v, (E + p) * u]
    Fy = [rho * v, rho * u * v, rho * v * v + p, (E + p) * v]
    out = []
    for a, b in zip(Fx, Fy):
        ga = torch.autograd.grad(a.sum(), x, retain_graph=True)[0]
        gb = torch.autograd.grad(b.sum(), y, retain_graph=True)[0]
        out.append(ga + gb)
    return torch.stack(out)


def _truncation_error(N, lim, eps2):
    Xe = torch.tensor(_mapped_nodes(N, extra=2))
    Xi = Xe[:, 2:-2, 2:-2]
    (S, vol) = metrics.metrics(Xi)
    xc = 0.25 * (Xe[:, :-1, :-1] + Xe[:, 1:, :-1] + Xe[:, :-1, 1:] + Xe[:, 1:, 1:])
    qpad = _ms_prims(xc[0], xc[1])
    case = synth.gaussian_bump_periodic(N, N, limiter=lim)
    case.scheme.lim_eps = [math.sqrt(eps2)] * 4
    P = Problem(case)
    R = P.block_residual_padded(qpad, S, vol)
    div = _exact_divergence(xc[0, 2:-2, 2:-2], xc[1, 2:-2, 2:-2])
    return (R - div).abs().amax(dim=(1, 2)).max().item()


@pytest.mark.parametrize("lim,min_order", [("none", 1.9), ("vanalbada", 1.8)])
def test_mms_truncation_order(lim, min_order):
    e = [_truncation_error(N, lim, 1e-4) for N in (16, 32, 64)]
    o1, o2 = math.log2(e[0] / e[1]), math.log2(e[1] / e[2])
    assert o2 > min_order and o2 < 2.2, (e, o1, o2)


# -- oblique shock -----------------------------------------------------------

@pytest.mark.slow
def test_oblique_shock_plateau():
    ref = json.load(open(os.path.join(HERE, "golden", "oblique_shock_M2p5_10deg.json")))
    ni, nj = 60, 40
    c = synth.compression_ramp(ni, nj)
    P = Problem(c)
    met = P.metrics()
    Q = P.initial_state()
    for _ in range(700):
        Q, _ = P.rk_step(Q, met)
    q = gas.prim_from_cons(Q[0], P.gamma)
    X = torch.tensor(c.blocks[0].nodes)
    xc = 0.25 * (X[0, :-1, :-1] + X[0, 1:, :-1] + X[0, :-1, 1:] + X[0, 1:, 1:])
    yc = 0.25 * (X[1, :-1, :-1] + X[1, 1:, :-1] + X[1, :-1, 1:] + X[1, 1:, 1:])
    yw = (xc - 0.5) * math.tan(math.radians(10.0))
    beta = math.radians(ref["beta_deg"])
    # cells well behind the shock and off the wall, away from the outflow
    shock_y = (xc - 0.5) * math.tan(beta)
    mask = (xc > 0.9) & (xc < 1.35) & (yc > yw + 0.05) & (yc < shock_y - 0.08)
    assert mask.sum() > 20
    p_ratio = (q[3][mask] / (1 / 1.4)).mean().item()
    r_ratio = q[0][mask].mean().item()
    assert p_ratio == pytest.approx(ref["p2_p1"], rel=0.02)
    assert r_ratio == pytest.approx(ref["rho2_rho1"], rel=0.02)
    # and the free stream ahead of the shock is untouched
    ahead = (yc > (xc - 0.5).clamp(min=0) * math.tan(beta) + 0.2)
    assert (q[3][ahead] / (1 / 1.4) - 1).abs().max() < 1e-6


# -- local time stepping and residual norms ------------------------------------

def test_local_stepping_equals_global_for_uniform_cell_steps():
    """On a uniform Cartesian periodic grid with uniform velocity and sound
    speed every cell has the same Omega/lambda, so local and global stepping
    take the same step and give the same state."""
    c = synth.gaussian_bump_periodic(16, 12, seed=3)
    # uniform u and p: every cell has the same sound speed and Omega/lambda
    # (up to the rounding of the node-based metrics)
    c = uniform(c, [1.0, 0.5, 0.0, 1 / 1.4])
    c.prims[0][0] *= 1.0 + 0.01 * np.sin(np.arange(16) * 0.7)[None, :]
    c.prims[0][3] = c.prims[0][0] / 1.4  # constant temperature: uniform c
    Pg = Problem(c)
    cl = copy.deepcopy(c)
    cl.scheme.local_dt = True
    Pl = Problem(cl)
    Q = Pg.initial_state()
    met = Pg.metrics()
    dl = Pl.local_steps(Q, met)[0]
    dg = float(Pg.time_step(Q, met))
    assert (dl - dg).abs().max() <= 1e-15 * dg
    Qg, dtg = Pg.rk_step(Q, met)
    Ql, dtl = Pl.rk_step(Q, met)
    assert (Qg[0] - Ql[0]).abs().max() <= 1e-14 and abs(float(dtg) - float(dtl)) <= 1e-15 * dg
    # and a state whose cells have different steps moves differently
    c2 = copy.deepcopy(c)
    c2.prims[0][3] = np.full_like(c2.prims[0][3], 1 / 1.4)
    P2g, P2l = Problem(c2), Problem(copy.deepcopy(cl))
    P2l.case.prims[0] = c2.prims[0]
    Q2 = P2g.initial_state()
    assert (P2g.rk_step(Q2, met)[0][0] - P2l.rk_step(Q2, met)[0][0]).abs().max() > 1e-9


def test_local_steps_follow_cell_size():
    """Cartesian closed form per cell: dt_i = CFL h_x h_y / (|u| h_y + c h_y + c h_x)
    with different spacings in the two halves of a stretched grid."""
    c = synth.compression_ramp(12, 8)
    c.blocks[0].nodes = synth.cartesian_nodes_2d(12, 8, lx=1.5)
    c.scheme.local_dt = True
    P = Problem(c)
    Q = P.initial_state()
    dts = P.local_steps(Q)[0]
    hx, hy = 1.5 / 12, 1.0 / 8
    u, cs = 2.5, 1.0
    ref = 0.5 * hx * hy / ((u + cs) * hy + cs * hx)
    assert (dts - ref).abs().max() <= 1e-15


def test_residual_norms_are_rms_per_variable():
    c = synth.jittered_periodic_square(10, 8, seed=6)
    P = Problem(c)
    Q = P.initial_state()
    N = P.residual_norms(Q)
    R = P.residual(Q)[0].reshape(4, -1)
    for v in range(4):
        ref = math.sqrt(sum(float(x) ** 2 for x in R[v]) / R.shape[1])
        assert abs(float(N[v]) - ref) <= 1e-14 * ref
