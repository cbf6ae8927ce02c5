"""GPU checks at the full workload sizes.

The oracle computes what it can at full size (single residuals of the 2D
workloads and of the 64-block patchwork); for the 256^3 box it computes the
residual of sampled sub-boxes one by one (ghosts by periodic wrap of the
oracle's own state); multi-step runs at full size are checked by properties
that hold at any size (conservation on periodic grids, undisturbed free
stream ahead of the ramp shock, bitwise agreement of launch modes) and by
finite differences of the HIP forward path for the unrolled gradient."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import gas, metrics
from parity_util import compare_residual, oracle_residual, q_ref, residual_scale

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _solver(case, **kw):
    from paper_2012_02925_amd.solver import Solver
    return Solver.from_case(case, device="cuda:0", **kw)


def test_ramp_1024_residual():
    _say("case: ramp 1024x1024 residual")
    case = synth.compression_ramp(1024, 1024)
    s = _solver(case)
    _, _, Rref = oracle_residual(case)
    qr = q_ref(case)
    ok, rep = compare_residual(s.residual(), Rref, qr, residual_scale(case, qr))
    _say("  ", rep)
    assert ok, rep


def test_ramp_1024_freestream_ahead_of_shock_after_500_steps():
    _say("case: ramp 1024x1024, 500 steps")
    case = synth.compression_ramp(1024, 1024)
    s = _solver(case)
    s.rk_step(500)
    Q = s.get_state().cpu().reshape(4, 1024, 1024)
    assert torch.isfinite(Q).all()
    q = gas.prim_from_cons(Q, 1.4)
    X = case.blocks[0].nodes
    xc = 0.25 * (X[0, :-1, :-1] + X[0, 1:, :-1] + X[0, :-1, 1:] + X[0, 1:, 1:])
    yc = 0.25 * (X[1, :-1, :-1] + X[1, 1:, :-1] + X[1, :-1, 1:] + X[1, 1:, 1:])
    # the corner disturbance cannot travel upstream of the Mach line from the corner
    mu = np.arcsin(1 / 2.5)
    ahead = torch.tensor((xc < 0.5 - 0.02) | (yc > (xc - 0.5) * np.tan(mu) + 0.05))
    free = torch.tensor([1.0, 2.5, 0.0, 1 / 1.4]).reshape(4, 1)
    dev = (q[:, ahead] - free).abs().max().item()
    _say("   max deviation ahead of the Mach line", dev)
    assert dev <= 1e-12
    # and the ramp has compressed the flow near the corner
    assert q[3].max() > 1.5 / 1.4


def _wrap_padded(q, i0, j0, k0, n, size):
    """Padded (size+4)^3 window of a periodic n^3 primitive field (oracle side)."""
    ii = (torch.arange(i0 - 2, i0 + size + 2) % n)
    jj = (torch.arange(j0 - 2, j0 + size + 2) % n)
    kk = (torch.arange(k0 - 2, k0 + size + 2) % n)
    return q[:, kk][:, :, jj][:, :, :, ii]


def test_box_256_residual_sampled():
    _say("case: jittered box 256^3 residual, sampled sub-boxes")
    n = 256
    case = synth.jittered_periodic_box(n=n, seed=0)
    s = _solver(case)
    R = s.residual().cpu().reshape(5, n, n, n)
    P = oracle.Problem(case)
    q = gas.prim_from_cons(gas.cons_from_prim(torch.tensor(case.prims[0]), 1.4), 1.4)
    X = torch.tensor(case.blocks[0].nodes)
    qr = q_ref(case)
    rng = np.random.default_rng(0)
    starts = [(0, 0, 0), (240, 240, 240), (0, 128, 240)] + [tuple(rng.integers(0, n - 16, 3)) for _ in range(3)]
    size = 16
    for (i0, j0, k0) in starts:
        qpad = _wrap_padded(q, i0, j0, k0, n, size)
        S, vol = metrics.metrics(X[:, k0:k0 + size + 1, j0:j0 + size + 1, i0:i0 + size + 1])
        Rref = P.block_residual_padded(qpad, S, vol)
        Rg = R[:, k0:k0 + size, j0:j0 + size, i0:i0 + size]
        # reference residual scale of the sub-box (see parity_util): flux of the
        # reference state through all faces of a cell without cancellation
        tot = torch.zeros_like(vol)
        for d in range(3):
            A = torch.sqrt((S[d] * S[d]).sum(0))
            ax = 2 - d
            tot = tot + A.narrow(ax, 0, size) + A.narrow(ax, 1, size)
        rs = torch.tensor(qr) * (qr[1] / qr[0] + 1.0) * float((tot / vol).max())
        ok, rep = compare_residual(Rg.reshape(5, -1), Rref.reshape(5, -1), qr, rs)
        _say("   box at", (i0, j0, k0), rep["rel_to_scale"], rep["guard"])
        assert ok, ((i0, j0, k0), rep)


def test_box_256_conservation_50_steps():
    _say("case: jittered box 256^3, 50 steps, conservation")
    n = 256
    case = synth.jittered_periodic_box(n=n, seed=0)
    s = _solver(case)
    Q0 = s.get_state().cpu()
    s.rk_step(50)
    Q1 = s.get_state().cpu()
    assert torch.isfinite(Q1).all()
    _, vol = metrics.metrics(case.blocks[0].nodes)
    vol = vol.reshape(-1)
    m0 = (Q0 * vol).sum(dim=1)
    m1 = (Q1 * vol).sum(dim=1)
    scale = (Q0.abs() * vol).sum(dim=1)
    drift = ((m1 - m0).abs() / scale).max().item()
    _say("   relative drift of the conserved totals", drift)
    assert drift <= 1e-12


def test_patchwork_64_blocks_residual_and_modes():
    _say("case: patchwork 64 blocks residual")
    case = synth.patchwork(seed=0)
    s = _solver(case)
    _, _, Rref = oracle_residual(case)
    qr = q_ref(case)
    ok, rep = compare_residual(s.residual(), Rref, qr, residual_scale(case, qr))
    _say("  ", rep)
    assert ok, rep
    # 200 steps: conservation, and per-block launches give the same bits
    s.rk_step(200)
    Qb = s.get_state().cpu()
    s2 = _solver(case)
    s2.set_exec("per_block", False)
    s2.rk_step(200)
    assert torch.equal(s2.get_state().cpu(), Qb)
    # equal cell volumes (uniform spacing in every block): plain sums are the
    # conserved totals; the y-momentum starts at zero, so momentum drifts are
    # measured against the x-momentum total
    Q0 = torch.cat([gas.cons_from_prim(torch.tensor(p), 1.4).reshape(4, -1) for p in case.prims], dim=1)
    scale = Q0.abs().sum(dim=1)
    scale[1:3] = scale[1:3].max()
    drift = ((Qb.sum(dim=1) - Q0.sum(dim=1)).abs() / scale).max().item()
    _say("   relative drift", drift)
    assert drift <= 1e-12


def _adjoint_case(n, dt):
    eps = 1e-2
    return synth.compression_ramp(n, n, limiter="vanalbada", lim_eps=[eps, eps, eps, eps / 1.4], dt_fixed=dt)


def test_ramp_512_vjp_matches_oracle():
    _say("case: ramp 512x512 residual VJP")
    case = _adjoint_case(512, 2e-4)
    rng = np.random.default_rng(1)
    case.prims[0] = case.prims[0] * (1 + 0.02 * rng.standard_normal(case.prims[0].shape))
    s = _solver(case, adjoint=True)
    P = oracle.Problem(case, requires_grad=True)
    Q = [x.detach().requires_grad_(True) for x in P.initial_state()]
    s.set_state(Q[0].detach().reshape(4, -1).to("cuda:0"))
    Rbar = torch.tensor(rng.standard_normal((4, case.ncells)))
    Qb, Xb, Tb = s.residual_vjp(Rbar.to("cuda:0"), nodes=True, inflow=True)
    R = P.residual(Q)[0].reshape(4, -1)
    gQ, gX, gT = torch.autograd.grad((R * Rbar).sum(), [Q[0], P.nodes[0], P.bc_params[0]])
    for name, a, b in (("Q", Qb, gQ.reshape(4, -1)), ("X", Xb, gX.reshape(2, -1)), ("theta", Tb[0], gT)):
        err = (a.cpu() - b).abs().max().item()
        ref = b.abs().max().item()
        _say("   %s err %.3e ref %.3e" % (name, err, ref))
        assert err <= 1e-10 * ref


def test_ramp_512_unrolled_gradient_vs_central_differences():
    """20 seeded directions (10 unit inflow-state directions, 10 smooth node
    displacement fields with largest component 1), central differences with
    h = 1e-7 of the HIP forward J against the adjoint, 1e-6 relative."""
    from paper_2012_02925_amd.autograd import unrolled_wall_pressure
    _say("case: ramp 512x512, 50 steps, FD vs adjoint")
    n, steps = 512, 50
    probe = _solver(synth.compression_ramp(n, n, limiter="vanalbada"))
    dt = probe.time_step().item()
    probe.close()
    case = _adjoint_case(n, dt)
    s = _solver(case, adjoint=True)
    theta0 = torch.tensor(case.meta["inflow"])
    nodes0 = torch.tensor(case.blocks[0].nodes).reshape(2, -1).to("cuda:0")
    th = theta0.clone().requires_grad_(True)
    X = nodes0.clone().requires_grad_(True)
    J = unrolled_wall_pressure(s, th, X, steps, every=10)
    J.backward()
    gT, gX = th.grad.clone(), X.grad.clone()

    def Jf(dth, dX):
        with torch.no_grad():
            return unrolled_wall_pressure(s, theta0 + dth, nodes0 + dX, steps, every=10).item()

    h = 1e-7
    dirs_t = synth.inflow_directions(10, seed=11)
    dirs_x = synth.node_displacement_fields(case.blocks[0], 10, seed=12)
    worst = 0.0
    for m in range(10):
        d = torch.tensor(dirs_t[m])
        fd = (Jf(h * d, 0.0) - Jf(-h * d, 0.0)) / (2 * h)
        ad = (gT * d).sum().item()
        rel = abs(fd - ad) / abs(fd)
        worst = max(worst, rel)
        _say("   inflow dir %d: fd %.12e ad %.12e rel %.2e" % (m, fd, ad, rel))
        assert rel <= 1e-6
    for m in range(10):
        d = torch.tensor(dirs_x[m]).reshape(2, -1).to("cuda:0")
        fd = (Jf(0.0, h * d) - Jf(0.0, -h * d)) / (2 * h)
        ad = (gX * d).sum().item()
        rel = abs(fd - ad) / abs(fd)
        worst = max(worst, rel)
        _say("   node dir %d: fd %.12e ad %.12e rel %.2e" % (m, fd, ad, rel))
        assert rel <= 1e-6
    _say("   worst relative disagreement", worst)
