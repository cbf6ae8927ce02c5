"""GPU adjoint: the hand-written residual VJP and the checkpointed unrolled
gradient against the oracle's automatic differentiation and against central
finite differences of the HIP forward path."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import gas

pytestmark = pytest.mark.gpu

VJP_TOL = 1e-10  # normwise: max|d| <= tol * max|ref| per output and variable


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _solver(case):
    from paper_2012_02925_amd.solver import Solver
    return Solver.from_case(case, device="cuda:0", adjoint=True)


def _ramp(ni=40, nj=26, lim="vanalbada", eps=1e-2, seed=0, dt=None):
    c = synth.compression_ramp(ni, nj, limiter=lim, lim_eps=[eps, eps, eps, eps / 1.4], dt_fixed=dt)
    rng = np.random.default_rng(seed)
    c.prims[0] = c.prims[0] * (1 + 0.03 * rng.standard_normal(c.prims[0].shape))
    return c


def _oracle_vjp(case, Rbar_packed):
    P = oracle.Problem(case, requires_grad=True)
    Q = [q.detach().requires_grad_(True) for q in P.initial_state()]
    R = P.residual(Q)
    Rflat = torch.cat([r.reshape(case.nvar, -1) for r in R], dim=1)
    leaves = Q + P.nodes + P.bc_params
    g = torch.autograd.grad((Rflat * Rbar_packed).sum(), leaves, allow_unused=True)
    nb = len(Q)
    Qbar = torch.cat([x.reshape(case.nvar, -1) for x in g[:nb]], dim=1)
    Xbar = torch.cat([x.reshape(case.dim, -1) for x in g[nb:2 * nb]], dim=1)
    Tbar = g[2 * nb:]
    return Qbar, Xbar, Tbar


def _close(a, b, tol, what):
    a = a.detach().cpu()
    b = b.detach().cpu()
    err = (a - b).abs().max().item()
    ref = b.abs().max().item()
    _say("  %s: max err %.3e, max ref %.3e, rel %.3e" % (what, err, ref, err / max(ref, 1e-300)))
    assert err <= tol * ref, (what, err, ref)


def _conservative_from_prims(case):
    P = oracle.Problem(case)
    return torch.cat([Q.reshape(case.nvar, -1) for Q in P.initial_state()], dim=1)


@pytest.mark.parametrize("lim,ni,nj", [("vanalbada", 40, 26), ("vanleer", 40, 26), ("none", 40, 26),
                                       ("vanalbada", 33, 17)])
def test_residual_vjp_matches_oracle_ramp(lim, ni, nj):
    """33 x 17: the last two cells along each axis fall into different 16-wide
    tiles, so the wall/inflow/outflow transposes of those cells run in the
    separate boundary pass while the others run inside the tile pass."""
    _say("case: ramp %dx%d residual VJP" % (ni, nj), lim)
    case = _ramp(ni=ni, nj=nj, lim=lim)
    s = _solver(case)
    s.set_state(_conservative_from_prims(case).to("cuda:0"))
    rng = np.random.default_rng(1)
    Rbar = torch.tensor(rng.standard_normal((case.nvar, case.ncells)))
    Qb, Xb, Tb = s.residual_vjp(Rbar.to("cuda:0"), nodes=True, inflow=True)
    Qr, Xr, Tr = _oracle_vjp(case, Rbar)
    for v in range(case.nvar):
        _close(Qb[v], Qr[v], VJP_TOL, "Qbar[%d]" % v)
    for c in range(2):
        _close(Xb[c], Xr[c], VJP_TOL, "Xbar[%d]" % c)
    _close(Tb[0], Tr[0], VJP_TOL, "inflow bar")


def test_residual_vjp_matches_oracle_multiblock():
    _say("case: patchwork 3x2 residual VJP")
    case = synth.patchwork(seed=5, nbx=3, nby=2, side_lo=6, side_hi=20, h=1.0 / 40, limiter="vanalbada")
    case.scheme.lim_eps = [1e-2, 1e-2, 1e-2, 1e-2 / 1.4]
    s = _solver(case)
    s.set_state(_conservative_from_prims(case).to("cuda:0"))
    rng = np.random.default_rng(2)
    Rbar = torch.tensor(rng.standard_normal((case.nvar, case.ncells)))
    Qb, Xb, _ = s.residual_vjp(Rbar.to("cuda:0"), nodes=True)
    Qr, Xr, _ = _oracle_vjp(case, Rbar)
    for v in range(case.nvar):
        _close(Qb[v], Qr[v], VJP_TOL, "Qbar[%d]" % v)
    for c in range(2):
        _close(Xb[c], Xr[c], VJP_TOL, "Xbar[%d]" % c)


@pytest.mark.parametrize("ni,nj", [(2, 17), (17, 2), (3, 33)])
def test_residual_vjp_thin_periodic_blocks(ni, nj):
    """Residual VJP on periodic blocks two or three cells thin (a block of 17
    or 33 cells also leaves its last cell alone in a 16-wide tile, so those
    cells go through the boundary pass): Q-bar and node cotangents against the
    oracle's autograd."""
    _say("case: thin periodic block %dx%d residual VJP" % (ni, nj))
    case = synth.jittered_periodic_square(ni, nj, seed=16, limiter="vanalbada")
    case.scheme.lim_eps = [1e-2, 1e-2, 1e-2, 1e-2 / 1.4]
    s = _solver(case)
    s.set_state(_conservative_from_prims(case).to("cuda:0"))
    rng = np.random.default_rng(3)
    Rbar = torch.tensor(rng.standard_normal((case.nvar, case.ncells)))
    Qb, Xb, _ = s.residual_vjp(Rbar.to("cuda:0"), nodes=True)
    Qr, Xr, _ = _oracle_vjp(case, Rbar)
    for v in range(case.nvar):
        _close(Qb[v], Qr[v], VJP_TOL, "Qbar[%d]" % v)
    for c in range(2):
        _close(Xb[c], Xr[c], VJP_TOL, "Xbar[%d]" % c)


def test_residual_vjp_reversed_connection():
    _say("case: reversed 2-block connection residual VJP")
    base = synth.jittered_periodic_square(20, 14, seed=8, limiter="vanleer")
    sp = synth.split_block_case(base, [9], [])
    A, B = sp.blocks
    Bn = synth.Block(B.ni, B.nj, 1, B.nodes[:, ::-1, ::-1].copy())
    nj = A.nj
    conns = [synth.Connection(0, synth.IMAX, [0], [nj], 1, synth.IMAX, [0], [nj], 1),
             synth.Connection(0, synth.IMIN, [0], [nj], 1, synth.IMIN, [0], [nj], 1),
             synth.Connection(0, synth.JMIN, [0], [A.ni], 0, synth.JMAX, [0], [A.ni], 0),
             synth.Connection(1, synth.JMIN, [0], [B.ni], 1, synth.JMAX, [0], [B.ni], 0)]
    case = synth.Case("rev", 2, [A, Bn], [], conns, [sp.prims[0], sp.prims[1][:, ::-1, ::-1].copy()],
                      base.scheme, 1)
    s = _solver(case)
    s.set_state(_conservative_from_prims(case).to("cuda:0"))
    rng = np.random.default_rng(3)
    Rbar = torch.tensor(rng.standard_normal((case.nvar, case.ncells)))
    Qb, Xb, _ = s.residual_vjp(Rbar.to("cuda:0"), nodes=True)
    Qr, Xr, _ = _oracle_vjp(case, Rbar)
    for v in range(case.nvar):
        _close(Qb[v], Qr[v], VJP_TOL, "Qbar[%d]" % v)
    _close(Xb, Xr, VJP_TOL, "Xbar")


def test_residual_vjp_dot_product_with_gpu_fd():
    """<Qbar, v> against central differences of the HIP residual itself."""
    case = _ramp(64, 40)
    s = _solver(case)
    Q0 = _conservative_from_prims(case).to("cuda:0")
    rng = np.random.default_rng(4)
    Rbar = torch.tensor(rng.standard_normal((case.nvar, case.ncells))).to("cuda:0")
    s.set_state(Q0)
    Qb, _, _ = s.residual_vjp(Rbar)
    h = 1e-7
    for trial in range(3):
        v = torch.tensor(rng.standard_normal(Q0.shape)).to("cuda:0") * Q0.abs().amax(dim=1, keepdim=True)
        s.set_state(Q0 + h * v)
        Rp = s.residual().clone()
        s.set_state(Q0 - h * v)
        Rm = s.residual().clone()
        fd = ((Rp - Rm) * Rbar).sum().item() / (2 * h)
        ad = (Qb * v).sum().item()
        _say("  trial", trial, fd, ad)
        assert abs(fd - ad) <= 1e-6 * abs(fd)


@pytest.mark.parametrize("stages", [1, 2, 4])
def test_rk_step_vjp_matches_oracle(stages):
    _say("case: ramp 30x20, one RK step VJP,", stages, "stages")
    case = _ramp(30, 20, dt=2e-3)
    case.scheme.rk_stages = stages
    s = _solver(case)
    s.set_state(_conservative_from_prims(case).to("cuda:0"))
    rng = np.random.default_rng(5)
    Gbar = torch.tensor(rng.standard_normal((case.nvar, case.ncells)))
    s.adjoint_reset()
    Qb = Gbar.clone().to("cuda:0").contiguous()
    s.rk_step_vjp(Qb)
    Xb, Tb = s.adjoint_result()
    # oracle
    P = oracle.Problem(case, requires_grad=True)
    Q = [q.detach().requires_grad_(True) for q in P.initial_state()]
    met = P.metrics()
    Q1, _ = P.rk_step(Q, met)
    g = torch.autograd.grad((Q1[0].reshape(case.nvar, -1) * Gbar).sum(), [Q[0], P.nodes[0], P.bc_params[0]])
    _close(Qb, g[0].reshape(case.nvar, -1), VJP_TOL, "Qbar")
    _close(Xb, g[1].reshape(2, -1), VJP_TOL, "Xbar")
    _close(Tb[0], g[2], VJP_TOL, "inflow bar")


def _oracle_unrolled_grad(case, steps):
    theta0 = torch.tensor(case.meta["inflow"])
    th = theta0.clone().requires_grad_(True)
    P = oracle.Problem(case, requires_grad=True)
    P.bc_params[0] = th
    met = P.metrics()
    q = th.reshape((-1,) + (1,) * case.dim).expand(case.prims[0].shape)
    Q = [gas.cons_from_prim(q, P.gamma)]
    for _ in range(steps):
        Q, _ = P.rk_step(Q, met)
    J = P.wall_pressure_integral(Q, met)
    gT, gX = torch.autograd.grad(J, [th, P.nodes[0]])
    return J.item(), gT, gX


def test_unrolled_gradient_matches_oracle():
    from paper_2012_02925_amd.autograd import unrolled_wall_pressure
    _say("case: ramp 36x24, 12 steps, checkpoints every 5")
    case = _ramp(36, 24, dt=2e-3)
    steps = 12
    Jr, gTr, gXr = _oracle_unrolled_grad(case, steps)
    s = _solver(case)
    theta = torch.tensor(case.meta["inflow"], requires_grad=True)
    nodes = torch.tensor(case.blocks[0].nodes).reshape(2, -1).to("cuda:0").requires_grad_(True)
    J = unrolled_wall_pressure(s, theta, nodes, steps, every=5)
    J.backward()
    _say("  J gpu %.15e oracle %.15e" % (J.item(), Jr))
    assert abs(J.item() - Jr) <= 1e-12 * abs(Jr)
    _close(theta.grad, gTr, VJP_TOL, "dJ/dtheta")
    _close(nodes.grad, gXr.reshape(2, -1), VJP_TOL, "dJ/dX")


def test_unrolled_gradient_3d_matches_oracle():
    """The unrolled wall-pressure gradient on the 3D wall/inflow box (two slip
    walls, supersonic inflow, periodic k): J, dJ/dtheta and the 3D node
    gradient after 8 steps against the oracle's autograd."""
    from paper_2012_02925_amd.autograd import unrolled_wall_pressure
    _say("case: 3D wall/inflow box 10x9x8, 8 steps, checkpoints every 3")
    case = _wall_box_3d()
    case.scheme.dt_fixed = 2e-3
    case.meta["inflow"] = case.bcs[0].params
    steps = 8
    Jr, gTr, gXr = _oracle_unrolled_grad(case, steps)
    s = _solver(case)
    theta = torch.tensor(case.meta["inflow"], requires_grad=True)
    nodes = torch.tensor(case.blocks[0].nodes).reshape(3, -1).to("cuda:0").requires_grad_(True)
    J = unrolled_wall_pressure(s, theta, nodes, steps, every=3)
    J.backward()
    _say("  J gpu %.15e oracle %.15e" % (J.item(), Jr))
    assert abs(J.item() - Jr) <= 1e-12 * abs(Jr)
    _close(theta.grad, gTr, VJP_TOL, "dJ/dtheta")
    _close(nodes.grad, gXr.reshape(3, -1), VJP_TOL, "dJ/dX")


def test_checkpoint_interval_does_not_change_gradient():
    from paper_2012_02925_amd.autograd import unrolled_wall_pressure
    case = _ramp(30, 20, dt=2e-3)
    grads = []
    for every in (1, 4, 10):
        s = _solver(case)
        theta = torch.tensor(case.meta["inflow"], requires_grad=True)
        nodes = torch.tensor(case.blocks[0].nodes).reshape(2, -1).to("cuda:0").requires_grad_(True)
        J = unrolled_wall_pressure(s, theta, nodes, 10, every=every)
        J.backward()
        grads.append((theta.grad.clone(), nodes.grad.clone().cpu()))
    for g in grads[1:]:
        assert torch.equal(g[0], grads[0][0]) and torch.equal(g[1], grads[0][1])


@pytest.mark.parametrize("stages", [1, 4])
def test_recorded_step_matches_recomputed_step(stages):
    """cfd_rk_step_record advances the state like cfd_rk_step, and the VJP over
    its recorded stages equals the VJP that recomputes them, bit for bit."""
    _say("case: ramp 30x20, recorded vs recomputed step VJP,", stages, "stages")
    case = _ramp(30, 20, dt=2e-3)
    case.scheme.rk_stages = stages
    s = _solver(case)
    Q0 = _conservative_from_prims(case).to("cuda:0")
    rng = np.random.default_rng(6)
    Gbar = torch.tensor(rng.standard_normal((case.nvar, case.ncells))).to("cuda:0")
    # recompute path
    s.set_state(Q0)
    s.adjoint_reset()
    Qa = Gbar.clone()
    s.rk_step_vjp(Qa)
    Xa, Ta = s.adjoint_result()
    s.rk_step(1)
    Q1a = s.get_state().clone()
    # recorded path
    s.set_state(Q0)
    s.adjoint_reset()
    slots, per = s.stage_record_buffer(1)
    s.rk_step_record(slots)
    Q1b = s.get_state().clone()
    Qb = Gbar.clone()
    s.rk_step_vjp_recorded(slots, Qb)
    Xb, Tb = s.adjoint_result()
    assert torch.equal(Q1a, Q1b)
    assert torch.equal(Qa, Qb)
    assert torch.equal(Xa, Xb) and torch.equal(Ta, Tb)


def test_residual_vjp_matches_oracle_3d_box():
    """3D path (face and cell passes, connection transposes across all six
    faces, node gradient)."""
    _say("case: jittered box 12x10x9 residual VJP")
    case = synth.jittered_periodic_box(seed=4, dims=(12, 10, 9))
    case.scheme.lim_eps = [1e-2, 1e-2, 1e-2, 1e-2, 1e-2 / 1.4]
    s = _solver(case)
    s.set_state(_conservative_from_prims(case).to("cuda:0"))
    rng = np.random.default_rng(7)
    Rbar = torch.tensor(rng.standard_normal((case.nvar, case.ncells)))
    Qb, Xb, _ = s.residual_vjp(Rbar.to("cuda:0"), nodes=True)
    Qr, Xr, _ = _oracle_vjp(case, Rbar)
    for v in range(case.nvar):
        _close(Qb[v], Qr[v], VJP_TOL, "Qbar[%d]" % v)
    for c in range(3):
        _close(Xb[c], Xr[c], VJP_TOL, "Xbar[%d]" % c)


def _wall_box_3d(dims=(10, 9, 8), seed=6, mach=2.0):
    """3D jittered box with supersonic inflow at imin, extrapolation at imax,
    slip walls at jmin and jmax and a periodic k direction; the state is the
    inflow state plus seeded smooth perturbations."""
    ni, nj, nk = dims
    blk = synth.Block(ni, nj, nk, synth.jittered_periodic_nodes_3d(ni, nj, nk, seed, amp=0.08))
    theta = np.array([1.0, mach, 0.1, -0.05, 1.0 / synth.GAMMA])
    rng = np.random.default_rng(seed + 11)
    prim = theta[:, None, None, None] * (1.0 + 0.03 * rng.standard_normal((5, nk, nj, ni)))
    bcs = [synth.full_face_patch(3, blk, 0, synth.IMIN, synth.SUP_INFLOW, theta),
           synth.full_face_patch(3, blk, 0, synth.IMAX, synth.EXTRAP_OUTFLOW),
           synth.full_face_patch(3, blk, 0, synth.JMIN, synth.SLIP_WALL),
           synth.full_face_patch(3, blk, 0, synth.JMAX, synth.SLIP_WALL)]
    conns = [synth.periodic_self_connections(3, ni, nj, nk)[2]]
    sch = synth.Scheme(limiter="vanalbada", lim_eps=[1e-2, 1e-2, 1e-2, 1e-2, 1e-2 / 1.4])
    return synth.Case("wall_box_%dx%dx%d" % dims, 3, [blk], bcs, conns, [prim], sch, 1)


def test_residual_vjp_matches_oracle_3d_walls_inflow():
    """3D residual VJP through slip walls (mirror ghosts with their dJ/dS
    term), supersonic inflow (dJ/dtheta), extrapolation and a periodic
    direction: Q-bar, node and inflow cotangents against the oracle."""
    _say("case: 3D wall/inflow box 10x9x8 residual VJP")
    case = _wall_box_3d()
    s = _solver(case)
    s.set_state(_conservative_from_prims(case).to("cuda:0"))
    rng = np.random.default_rng(8)
    Rbar = torch.tensor(rng.standard_normal((case.nvar, case.ncells)))
    Qb, Xb, Tb = s.residual_vjp(Rbar.to("cuda:0"), nodes=True, inflow=True)
    Qr, Xr, Tr = _oracle_vjp(case, Rbar)
    for v in range(case.nvar):
        _close(Qb[v], Qr[v], VJP_TOL, "Qbar[%d]" % v)
    for c in range(3):
        _close(Xb[c], Xr[c], VJP_TOL, "Xbar[%d]" % c)
    _close(Tb[0], Tr[0], VJP_TOL, "inflow bar")


def test_node_gradient_3d_matches_gpu_finite_difference():
    """<Rbar, dR/dX . dX> from the 3D node gradient against a central
    difference of the HIP forward residual along a smooth node displacement
    (the forward path and its transpose agree, independently of the oracle)."""
    from paper_2012_02925_amd.solver import Solver
    case = _wall_box_3d(dims=(9, 8, 7), seed=2)
    s = _solver(case)
    Q0 = _conservative_from_prims(case).to("cuda:0")
    s.set_state(Q0)
    rng = np.random.default_rng(5)
    Rbar = torch.tensor(rng.standard_normal((case.nvar, case.ncells)))
    _, Xb, _ = s.residual_vjp(Rbar.to("cuda:0"), nodes=True)
    s.close()
    blk = case.blocks[0]
    ni, nj, nk = blk.ni, blk.nj, blk.nk
    z, y, x = np.meshgrid(*[np.arange(n + 1) / n for n in (nk, nj, ni)], indexing="ij")
    dX = np.stack([np.sin(2 * np.pi * (x + 0.3 * y)) * np.cos(np.pi * z),
                   np.cos(2 * np.pi * (y - 0.2 * z)) * np.sin(np.pi * x),
                   np.sin(np.pi * (x + y + z))]) * (0.2 / ni)
    lin = float((Xb.cpu() * torch.tensor(dX.reshape(3, -1))).sum())
    vals = []
    for sign in (1.0, -1.0):
        h = 1e-6
        c2 = _wall_box_3d(dims=(9, 8, 7), seed=2)
        c2.blocks[0] = synth.Block(ni, nj, nk, blk.nodes + sign * h * dX)
        s2 = Solver.from_case(c2, device="cuda:0")
        s2.set_state(Q0)
        vals.append(float((s2.residual().cpu() * Rbar).sum()))
        s2.close()
    fd = (vals[0] - vals[1]) / (2 * 1e-6)
    _say("  <Xbar, dX> %.12e   central difference %.12e" % (lin, fd))
    assert abs(lin - fd) <= 1e-6 * max(abs(lin), 1e-300)


def test_residual_fn_forward_backward_and_state_kept():
    """ResidualFn (torch.autograd.Function over cfd_residual / cfd_residual_vjp):
    forward equals cfd_residual at Q, torch.autograd.grad through it equals the
    oracle's autograd VJP, and the solver's own state is unchanged by both
    passes (bit for bit)."""
    from paper_2012_02925_amd.autograd import ResidualFn
    _say("case: ramp 40x26, ResidualFn")
    case = _ramp(40, 26, seed=4)
    s = _solver(case)
    held = s.get_state().clone()  # the solver's state: the case's initial state
    Q = _conservative_from_prims(_ramp(40, 26, seed=5)).to("cuda:0").requires_grad_(True)
    R = ResidualFn.apply(Q, s)
    torch.cuda.synchronize()
    assert torch.equal(s.get_state(), held)
    # forward = cfd_residual at Q
    from paper_2012_02925_amd.solver import Solver
    s2 = Solver.from_case(case, device="cuda:0", adjoint=True)
    s2.set_state(Q.detach())
    assert torch.equal(R.detach(), s2.residual())
    rng = np.random.default_rng(6)
    Rbar = torch.tensor(rng.standard_normal((case.nvar, case.ncells)))
    (g,) = torch.autograd.grad(R, Q, grad_outputs=Rbar.to("cuda:0"))
    torch.cuda.synchronize()
    assert torch.equal(s.get_state(), held)
    case_q = _ramp(40, 26, seed=5)
    Qr, _, _ = _oracle_vjp(case_q, Rbar)
    for v in range(case.nvar):
        _close(g[v], Qr[v], VJP_TOL, "ResidualFn grad Q[%d]" % v)
    s.close()
    s2.close()


def test_rk_step_record_matches_rk_step_navier_stokes():
    """cfd_rk_step_record advances exactly like cfd_rk_step, also with the
    viscous residual recomputed for every stage input (laminar Navier-Stokes),
    and leaves the ghost-filled stage inputs in the caller's slots."""
    from paper_2012_02925_amd.solver import Solver
    case = synth.jittered_periodic_square(48, 40, seed=3)
    case.scheme.viscosity = 0.01
    a = Solver.from_case(case, device="cuda:0")
    b = Solver.from_case(case, device="cuda:0")
    slots, per = b.stage_record_buffer(1)
    for _ in range(3):
        a.rk_step(1)
        b.rk_step_record(slots[:per])
    torch.cuda.synchronize()
    assert torch.equal(a.get_state(), b.get_state())
    a.close()
    b.close()
