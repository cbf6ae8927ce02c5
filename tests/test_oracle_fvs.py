"""Pins for the oracle's flux-vector splittings (van Leer, Steger-Warming), no GPU.

Each pin checks a property the splittings are defined by, independently of the
closed forms in oracle/fvs.py: the Steger-Warming parts against R diag(l+-)
R^-1 Q built from an eigendecomposition of the flux Jacobian (autograd of a
conservative flux written here), van Leer's parts against their defining
properties (F+ + F- = F, upwinding beyond Mach 1, value and slope continuity
at |M| = 1, a vanishing eigenvalue of dF+-/dQ for |M| < 1), and both against
consistency, rotation and freestream preservation / conservation in the
solver."""
import copy

import numpy as np
import pytest
import torch

import synth
from oracle import Problem, fvs, gas

G = 1.4


def flux_conservative(Q, n):
    """Normal flux written directly in conservative variables (test-local)."""
    rho = Q[0]
    vel = Q[1:-1] / rho
    E = Q[-1]
    p = (G - 1.0) * (E - 0.5 * rho * (vel * vel).sum())
    vn = (vel * n).sum()
    return torch.cat([(rho * vn)[None], rho * vel * vn + p * n, ((E + p) * vn)[None]])


def prim_of(Q):
    rho = Q[0]
    vel = Q[1:-1] / rho
    p = (G - 1.0) * (Q[-1] - 0.5 * rho * (vel * vel).sum())
    return torch.cat([rho[None], vel, p[None]])


def state(dim, rho, vn, vt, p, n):
    """Primitive state with normal velocity vn along unit n and tangential vt."""
    t = torch.zeros(dim, dtype=torch.float64)
    t[0], t[1] = -n[1], n[0]
    vel = vn * n + vt * t
    return torch.cat([torch.tensor([rho], dtype=torch.float64), vel, torch.tensor([p], dtype=torch.float64)])


def unit(dim, seed):
    v = torch.tensor(np.random.default_rng(seed).standard_normal(dim))
    return v / v.norm()


MACHS = [-2.3, -1.0, -0.6, -0.1, 0.0, 0.3, 0.9, 1.0, 1.7]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("which", ["vanleer", "sw"])
def test_split_sums_to_the_flux(dim, which):
    part = fvs.van_leer_part if which == "vanleer" else fvs.steger_warming_part
    n = unit(dim, 1)
    for M in MACHS:
        c = 1.1
        q = state(dim, 0.9, M * c, 0.4, c * c * 0.9 / G, n)
        Fp = part(q[:, None], n[:, None], G, 1.0)[:, 0]
        Fm = part(q[:, None], n[:, None], G, -1.0)[:, 0]
        Q = gas.cons_from_prim(q[:, None], G)[:, 0]
        F = flux_conservative(Q, n)
        assert torch.allclose(Fp + Fm, F, rtol=0, atol=1e-14 * F.abs().max().item() + 1e-15), (which, M)


@pytest.mark.parametrize("dim", [2, 3])
def test_steger_warming_matches_eigen_splitting(dim):
    """F+- = R diag(l+-) R^-1 Q with A_n = dF_n/dQ = R diag(l) R^-1."""
    n = unit(dim, 2)
    for M in MACHS:
        c = 0.8
        q = state(dim, 1.3, M * c, -0.25, c * c * 1.3 / G, n)
        Q = gas.cons_from_prim(q[:, None], G)[:, 0]
        A = torch.autograd.functional.jacobian(lambda X: flux_conservative(X, n), Q)
        lam, R = torch.linalg.eig(A)
        Rinv = torch.linalg.inv(R)
        for sign in (1.0, -1.0):
            lp = 0.5 * (lam.real + sign * lam.real.abs())
            ref = (R @ torch.diag(lp.to(R.dtype)) @ Rinv @ Q.to(R.dtype)).real
            got = fvs.steger_warming_part(q[:, None], n[:, None], G, sign)[:, 0]
            assert torch.allclose(got, ref, rtol=0, atol=1e-12 * Q.abs().max().item()), (M, sign)


@pytest.mark.parametrize("dim", [2, 3])
def test_van_leer_upwinding_and_continuity(dim):
    n = unit(dim, 3)
    c = 1.0
    rho, p = 1.0, 1.0 / G

    def parts(M):
        q = state(dim, rho, M * c, 0.3, p, n)[:, None]
        return fvs.van_leer_part(q, n[:, None], G, 1.0)[:, 0], fvs.van_leer_part(q, n[:, None], G, -1.0)[:, 0]

    for M in (1.0, 1.4, 3.0):
        Fp, Fm = parts(M)
        F = flux_conservative(gas.cons_from_prim(state(dim, rho, M * c, 0.3, p, n)[:, None], G)[:, 0], n)
        assert torch.allclose(Fp, F, atol=1e-14) and Fm.abs().max() == 0.0
        Fp, Fm = parts(-M)
        F = flux_conservative(gas.cons_from_prim(state(dim, rho, -M * c, 0.3, p, n)[:, None], G)[:, 0], n)
        assert torch.allclose(Fm, F, atol=1e-14) and Fp.abs().max() == 0.0
    # value and slope continuity at M = +-1 (one-sided differences from both sides)
    h = 1e-6
    for Ms in (1.0, -1.0):
        for k in (0, 1):
            lo, at, hi = parts(Ms - h)[k], parts(Ms)[k], parts(Ms + h)[k]
            assert (hi - lo).abs().max() < 1e-5
            dl, dr = (at - lo) / h, (hi - at) / h
            assert (dl - dr).abs().max() < 1e-4 * max(1.0, dl.abs().max().item())


@pytest.mark.parametrize("dim", [2, 3])
def test_van_leer_jacobians_have_a_zero_eigenvalue(dim):
    """van Leer's design requirement: for |M| < 1, dF+-/dQ has one vanishing
    eigenvalue and the rest of one sign (>= 0 for F+, <= 0 for F-)."""
    n = unit(dim, 4)
    for M in (-0.8, -0.3, 0.0, 0.45, 0.95):
        q = state(dim, 1.2, M * 0.9, 0.2, 0.9 * 0.9 * 1.2 / G, n)
        Q = gas.cons_from_prim(q[:, None], G)[:, 0]
        for sign in (1.0, -1.0):
            J = torch.autograd.functional.jacobian(
                lambda X: fvs.van_leer_part(prim_of(X)[:, None], n[:, None], G, sign)[:, 0], Q)
            ev = torch.linalg.eigvals(J).real
            assert ev.abs().min() < 1e-12 * ev.abs().max(), (M, sign, ev)
            assert (sign * ev).min() > -1e-10, (M, sign, ev)


@pytest.mark.parametrize("which", ["vanleer_fvs", "steger_warming"])
def test_flux_consistency_and_rotation(which):
    rng = np.random.default_rng(5)
    fn = fvs.van_leer_flux if which == "vanleer_fvs" else fvs.steger_warming_flux
    q = torch.tensor(np.vstack([rng.uniform(0.5, 2, 8), rng.uniform(-1.5, 1.5, (2, 8)), rng.uniform(0.3, 1.2, 8)]))
    S = torch.tensor(rng.standard_normal((2, 8)))
    F = fn(q, q, S, G)
    A = torch.sqrt((S * S).sum(0))
    ref = gas.normal_flux(q, S / A, G) * A
    assert torch.allclose(F, ref, rtol=1e-13, atol=1e-14)
    # rotation: rotate normals and velocities by 37 degrees
    qL = torch.tensor(np.vstack([rng.uniform(0.5, 2, 8), rng.uniform(-1.5, 1.5, (2, 8)), rng.uniform(0.3, 1.2, 8)]))
    th = np.deg2rad(37.0)
    Rm = torch.tensor([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    rot = lambda x: torch.cat([x[:1], Rm @ x[1:3], x[3:]])
    F1 = fn(qL, q, S, G)
    F2 = fn(rot(qL), rot(q), Rm @ S, G)
    assert torch.allclose(rot(F1), F2, rtol=1e-12, atol=1e-13)


def _uniform(case, prim):
    c = copy.deepcopy(case)
    for b, q in enumerate(c.prims):
        c.prims[b] = np.broadcast_to(np.asarray(prim, float).reshape([-1] + [1] * (q.ndim - 1)), q.shape).copy()
    return c


@pytest.mark.parametrize("which", ["vanleer_fvs", "steger_warming"])
def test_solver_freestream_and_conservation(which):
    c2 = synth.jittered_periodic_square(20, 16, seed=1, limiter="vanalbada")
    c2.scheme.flux = which
    P = Problem(_uniform(c2, [1.0, 0.7, -0.3, 1 / 1.4]))
    assert P.residual(P.initial_state())[0].abs().max() < 1e-12
    c3 = synth.jittered_periodic_box(dims=(8, 7, 6), seed=2)
    c3.scheme.flux = which
    P = Problem(c3)
    Q = P.initial_state()
    vol = P.metrics()[0][1]
    R = P.residual(Q)
    assert (R[0] * vol).sum(dim=(1, 2, 3)).abs().max() < 1e-14
    assert R[0].abs().max() > 1e-3  # a non-trivial residual
