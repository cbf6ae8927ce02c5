"""Pins for the oracle's derivatives (no GPU).

The oracle's gradients come from torch.autograd over the plain residual; these
tests tie them to central finite differences of the same function and to
forward-mode derivatives (dot-product test), so a detached or non-smooth term
would show up here."""
import numpy as np
import pytest
import torch

import synth
from oracle import Problem, gas


def small_ramp(ni=18, nj=12, eps=1e-2):
    # The van Albada regularisation sets the length scale of the limiter's
    # smooth corner at a = b = 0; central differences with step h resolve it
    # to about (h |v| / eps)^2, so eps = 1e-2 keeps h = 1e-7 differences at
    # about 1e-10 relative (eps = 1e-4 would limit them to about 1e-6).
    c = synth.compression_ramp(ni, nj, limiter="vanalbada", lim_eps=[eps, eps, eps, eps / 1.4])
    rng = np.random.default_rng(0)
    c.prims[0] = c.prims[0] * (1 + 0.03 * rng.standard_normal(c.prims[0].shape))
    return c


def test_residual_vjp_matches_central_fd():
    c = small_ramp()
    P = Problem(c, requires_grad=True)
    Q = [q.detach().requires_grad_(True) for q in P.initial_state()]
    R = P.residual(Q)
    rng = np.random.default_rng(1)
    Rbar = torch.tensor(rng.standard_normal(R[0].shape))
    gQ, gX, gT = torch.autograd.grad((R[0] * Rbar).sum(), [Q[0], P.nodes[0], P.bc_params[0]])

    def f(dQ=0.0, dX=0.0, dT=0.0):
        P2 = Problem(c)
        P2.nodes[0] = P2.nodes[0] + dX
        P2.bc_params[0] = P2.bc_params[0] + dT
        return (P2.residual([Q[0].detach() + dQ])[0] * Rbar).sum().item()

    h = 1e-7
    for trial in range(4):
        # directions scaled so the derivative is well above the FD round-off
        # (about 1e-16 |R| / h summed over the cells)
        vQ = torch.tensor(rng.standard_normal(Q[0].shape))
        vX = torch.tensor(rng.standard_normal(P.nodes[0].shape)) * 1e-2
        vT = torch.tensor(rng.standard_normal(4)) * 1e-1
        fd = (f(h * vQ, h * vX, h * vT) - f(-h * vQ, -h * vX, -h * vT)) / (2 * h)
        ad = (gQ * vQ).sum() + (gX * vX).sum() + (gT * vT).sum()
        assert abs(fd - ad.item()) <= 1e-6 * abs(fd), (trial, fd, ad)


def test_forward_and_reverse_mode_agree():
    c = small_ramp(14, 10)
    P = Problem(c)
    Q0 = P.initial_state()[0]
    rng = np.random.default_rng(2)
    v = torch.tensor(rng.standard_normal(Q0.shape))
    w = torch.tensor(rng.standard_normal(Q0.shape))
    met = P.metrics()
    fn = lambda Q: P.residual([Q], met)[0]
    _, jv = torch.func.jvp(fn, (Q0,), (v,))
    _, vjp = torch.func.vjp(fn, Q0)
    (jtw,) = vjp(w)
    a, b = (jv * w).sum().item(), (jtw * v).sum().item()
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_unrolled_objective_gradient_matches_fd():
    c = small_ramp(15, 10)
    c.scheme.dt_fixed = 2e-3
    steps = 6
    theta0 = torch.tensor(c.meta["inflow"])

    def J_of(theta, dX=0.0):
        P = Problem(c)
        P.bc_params[0] = theta
        P.nodes[0] = P.nodes[0] + dX
        met = P.metrics()
        shape = c.prims[0].shape
        q = theta.reshape(-1, 1, 1).expand(shape)
        Q = [gas.cons_from_prim(q, P.gamma)]
        for _ in range(steps):
            Q, _ = P.rk_step(Q, met)
        return P.wall_pressure_integral(Q, met)

    th = theta0.clone().requires_grad_(True)
    dX = torch.zeros(c.blocks[0].nodes.shape, requires_grad=True)
    J = J_of(th, dX)
    gT, gX = torch.autograd.grad(J, [th, dX])
    rng = np.random.default_rng(3)
    h = 1e-7
    for trial in range(3):
        vT = torch.tensor(rng.standard_normal(4)) * 1e-2
        vX = torch.tensor(rng.standard_normal(dX.shape)) * 1e-3
        fd = (J_of(theta0 + h * vT, h * vX) - J_of(theta0 - h * vT, -h * vX)).item() / (2 * h)
        ad = ((gT * vT).sum() + (gX * vX).sum()).item()
        assert abs(fd - ad) <= 1e-6 * abs(fd), (trial, fd, ad)
