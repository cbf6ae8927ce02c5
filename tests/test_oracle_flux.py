"""Pins for the oracle's gas relations and Roe flux (no GPU).

The Roe dissipation is checked against an independent construction: the
conservative flux Jacobian at the Roe-average state is formed by automatic
differentiation of a flux written here in conservative variables, diagonalised
with numpy, and |A~| (Q_R - Q_L) is compared with the oracle's dissipation.
"""
import math

import numpy as np
import pytest
import torch

from oracle import gas, roe

G = 1.4


def rand_prims(rng, dim, n, mach=0.7):
    rho = rng.uniform(0.5, 2.0, n)
    vel = rng.uniform(-mach, mach, (dim, n))
    p = rng.uniform(0.4, 1.5, n)
    return torch.tensor(np.vstack([rho, vel, p]))


def rand_S(rng, dim, n):
    return torch.tensor(rng.standard_normal((dim, n)))


def flux_conservative(Q, n):
    """Normal flux written directly in conservative variables (test-local)."""
    rho = Q[0]
    vel = Q[1:-1] / rho
    E = Q[-1]
    p = (G - 1.0) * (E - 0.5 * rho * (vel * vel).sum())
    vn = (vel * n).sum()
    return torch.cat([(rho * vn)[None], rho * vel * vn + p * n, ((E + p) * vn)[None]])


@pytest.mark.parametrize("dim", [2, 3])
def test_prim_cons_roundtrip(dim):
    q = rand_prims(np.random.default_rng(0), dim, 50)
    back = gas.prim_from_cons(gas.cons_from_prim(q, G), G)
    assert torch.allclose(back, q, rtol=1e-14, atol=0)


@pytest.mark.parametrize("dim", [2, 3])
def test_consistency_exact(dim):
    rng = np.random.default_rng(1)
    q = rand_prims(rng, dim, 40)
    S = rand_S(rng, dim, 40)
    A = torch.sqrt((S * S).sum(0))
    F = roe.roe_flux(q, q, S, G, efix=0.1)
    ref = A * gas.normal_flux(q, S / A, G)
    assert torch.equal(F, ref)


@pytest.mark.parametrize("dim", [2, 3])
def test_roe_property_signed_waves(dim):
    """With |lambda| replaced by lambda the wave sum equals F(qR) - F(qL)
    (Roe's property), so the flux collapses to the left flux."""
    rng = np.random.default_rng(2)
    qL, qR = rand_prims(rng, dim, 64), rand_prims(rng, dim, 64)
    S = rand_S(rng, dim, 64)
    A = torch.sqrt((S * S).sum(0))
    F = roe.roe_flux(qL, qR, S, G, absfn=lambda l: l)
    ref = A * gas.normal_flux(qL, S / A, G)
    assert torch.allclose(F, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("efix", [0.0, 0.1, 0.3])
def test_dissipation_matches_eigendecomposition(dim, efix):
    rng = np.random.default_rng(3 + dim)
    for trial in range(12):
        qL = rand_prims(rng, dim, 1)[:, 0]
        qR = rand_prims(rng, dim, 1)[:, 0]
        S = rand_S(rng, dim, 1)[:, 0]
        A = torch.sqrt((S * S).sum())
        n = S / A
        # Roe-average state written from its definition (sqrt(rho) weights)
        wL, wR = torch.sqrt(qL[0]), torch.sqrt(qR[0])
        HL = (G / (G - 1) * qL[-1] / qL[0] + 0.5 * (qL[1:-1] ** 2).sum())
        HR = (G / (G - 1) * qR[-1] / qR[0] + 0.5 * (qR[1:-1] ** 2).sum())
        rho_t = wL * wR
        u_t = (wL * qL[1:-1] + wR * qR[1:-1]) / (wL + wR)
        H_t = (wL * HL + wR * HR) / (wL + wR)
        p_t = (G - 1) / G * rho_t * (H_t - 0.5 * (u_t ** 2).sum())
        Qt = torch.cat([rho_t[None], rho_t * u_t, (p_t / (G - 1) + 0.5 * rho_t * (u_t ** 2).sum())[None]])
        Jac = torch.autograd.functional.jacobian(lambda Q: flux_conservative(Q, n), Qt).numpy()
        QL = gas.cons_from_prim(qL[:, None], G)[:, 0]
        QR = gas.cons_from_prim(qR[:, None], G)[:, 0]
        # Roe property: A~ (QR - QL) = F(QR) - F(QL)
        dF = (flux_conservative(QR, n) - flux_conservative(QL, n)).numpy()
        assert np.allclose(Jac @ (QR - QL).numpy(), dF, rtol=1e-11, atol=1e-11)
        # the repeated eigenvalue may come back as a complex pair split by
        # round-off: keep the decomposition complex and take the real part
        lam, V = np.linalg.eig(Jac)
        lr = lam.real
        c_t = 0.5 * (lr.max() - lr.min())
        delta = efix * c_t
        f = np.where(np.abs(lr) >= delta, np.abs(lr), (lr ** 2 + delta ** 2) / (2 * delta) if delta > 0 else 0)
        Dref = (V @ np.diag(f) @ np.linalg.solve(V, (QR - QL).numpy().astype(complex))).real
        F = roe.roe_flux(qL[:, None], qR[:, None], S[:, None], G, efix=efix)[:, 0] / A
        FL = gas.normal_flux(qL[:, None], n[:, None], G)[:, 0]
        FR = gas.normal_flux(qR[:, None], n[:, None], G)[:, 0]
        D = (FL + FR - 2.0 * F).numpy()
        assert np.allclose(D, Dref, rtol=1e-10, atol=1e-11), (trial, D, Dref)


def test_supersonic_upwinding():
    rng = np.random.default_rng(4)
    q = rand_prims(rng, 2, 30, mach=0.0)
    q[1] = 3.0 + torch.rand(30)  # |u| > c + delta everywhere
    q2 = q.clone()
    q2[0] *= 1.05
    q2[-1] *= 0.97
    S = torch.tensor([[1.0] * 30, [0.0] * 30])
    F = roe.roe_flux(q, q2, S, G, efix=0.1)
    assert torch.allclose(F, gas.normal_flux(q, S, G), rtol=1e-12)
    F = roe.roe_flux(q2, q, -S, G, efix=0.1)  # flow now toward the left state
    assert torch.allclose(F, -gas.normal_flux(q, S, G), rtol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_flip_and_rotation_invariance(dim):
    rng = np.random.default_rng(5)
    qL, qR = rand_prims(rng, dim, 20), rand_prims(rng, dim, 20)
    S = rand_S(rng, dim, 20)
    F = roe.roe_flux(qL, qR, S, G)
    Fb = roe.roe_flux(qR, qL, -S, G)
    assert torch.allclose(F, -Fb, rtol=1e-12, atol=1e-13)
    # rotate the frame
    M = torch.tensor(np.linalg.qr(rng.standard_normal((dim, dim)))[0])
    rot = lambda q: torch.cat([q[:1], M @ q[1:-1], q[-1:]])
    Fr = roe.roe_flux(rot(qL), rot(qR), M @ S, G)
    assert torch.allclose(torch.cat([Fr[:1], M.T @ Fr[1:-1], Fr[-1:]]), F, rtol=1e-12, atol=1e-13)


def test_harten_abs_is_c1():
    delta = torch.tensor(0.3)
    for x in (0.3, -0.3):
        lo = roe.harten_abs(torch.tensor(x * (1 - 1e-9)), delta)
        hi = roe.harten_abs(torch.tensor(x * (1 + 1e-9)), delta)
        assert abs(lo - hi) < 1e-9
        lam = torch.tensor(x * (1 - 1e-12), requires_grad=True)
        (g,) = torch.autograd.grad(roe.harten_abs(lam, delta), lam)
        assert abs(g.item() - math.copysign(1.0, x)) < 1e-9
    assert roe.harten_abs(torch.tensor(0.0), delta).item() == pytest.approx(0.15)
