"""Pins for the oracle's limiter freezing, no GPU.

The frozen factor is checked against closed forms derived by hand from the
limiters' slope forms (van Leer: the harmonic mean over the arithmetic mean;
van Albada: 2(ab + e^2)/(a^2 + b^2 + 2e^2)), the frozen face states against
the properties that define freezing (unchanged at the freeze state, linear in
the state afterwards, phi = 1 is the unlimited central scheme) and the solver
against them on 2D and 3D cases."""
import numpy as np
import pytest
import torch

import synth
from oracle import Problem, muscl


def rand_pairs(seed, n=4000):
    g = torch.Generator().manual_seed(seed)
    a = torch.randn(n, generator=g, dtype=torch.float64)
    b = torch.randn(n, generator=g, dtype=torch.float64)
    # exact zeros, equal values and opposite values
    a[:50] = 0.0
    b[50:100] = 0.0
    a[100:150] = b[100:150]
    a[150:200] = -b[150:200]
    a[200:210] = 0.0
    b[200:210] = 0.0
    return a, b


def test_frozen_factor_closed_forms():
    a, b = rand_pairs(1)
    phi = muscl.frozen_factor(a, b, "vanleer")
    ref = torch.where(a * b > 0, 4.0 * a * b / (a + b) ** 2, torch.zeros_like(a))
    assert torch.allclose(phi, ref, rtol=1e-14, atol=1e-15)
    assert float(phi.min()) >= 0.0 and float(phi.max()) <= 1.0 + 1e-15
    for e in (0.0, 1e-2, 0.3):
        e2 = torch.full_like(a, e * e)
        phi = muscl.frozen_factor(a, b, "vanalbada", e2)
        ref = 2.0 * (a * b + e * e) / (a * a + b * b + 2.0 * e * e)
        ref = torch.where(a + b == 0, torch.zeros_like(ref), ref)
        ref = torch.where((a == 0) & (b == 0), torch.zeros_like(ref), ref)
        # S(a, b) / ((a + b)/2) cancels where a ~ -b: its rounding error grows
        # like (|a| + |b|) / |a + b|, the closed form's does not
        cond = (a.abs() + b.abs()) / torch.where(a + b == 0, torch.ones_like(a), (a + b).abs())
        assert bool(((phi - ref).abs() <= 1e-14 * cond + 1e-15).all()), e
        assert float(phi.abs().max()) <= 1.0 + 1e-14


def padded_line(seed, n=12, nvar=4):
    g = torch.Generator().manual_seed(seed)
    return torch.randn(nvar, n + 4, generator=g, dtype=torch.float64)


@pytest.mark.parametrize("lim", ["vanleer", "vanalbada"])
def test_frozen_face_states_at_freeze_and_linear_after(lim):
    q = padded_line(3)
    e2 = torch.full((4, 1), 1e-4)
    Dm, Dp = muscl.cell_differences(q, 1)
    phi = muscl.frozen_factor(Dp, Dm, lim, e2)
    assert phi.shape == (4, 14)
    # unchanged at the freeze state, for any kappa
    for kappa in (-1.0, 0.0, 1.0 / 3.0):
        live = muscl.face_states(q, 1, lim, 1.0, kappa, e2)
        frozen = muscl.face_states(q, 1, lim, 1.0, kappa, e2, phi)
        for x, y in zip(live, frozen):
            assert torch.allclose(x, y, rtol=0, atol=1e-15)
    # afterwards the face states are linear in the state
    q1, q2 = padded_line(4), padded_line(5)
    f1 = muscl.face_states(q1, 1, lim, 1.0, -1.0, e2, phi)
    f2 = muscl.face_states(q2, 1, lim, 1.0, -1.0, e2, phi)
    f12 = muscl.face_states(q1 + 2.0 * q2, 1, lim, 1.0, -1.0, e2, phi)
    for x, y, z in zip(f1, f2, f12):
        assert torch.allclose(z, x + 2.0 * y, rtol=0, atol=1e-14)
    # ... and the live limiter is not
    g12 = muscl.face_states(q1 + 2.0 * q2, 1, lim, 1.0, -1.0, e2)
    g1 = muscl.face_states(q1, 1, lim, 1.0, -1.0, e2)
    g2 = muscl.face_states(q2, 1, lim, 1.0, -1.0, e2)
    assert float((g12[0] - g1[0] - 2.0 * g2[0]).abs().max()) > 1e-3


def test_unit_factor_is_the_central_scheme():
    q = padded_line(6)
    phi = torch.ones(4, 14, dtype=torch.float64)
    fz = muscl.face_states(q, 1, "vanleer", 1.0, -1.0, None, phi)
    fromm = muscl.face_states(q, 1, "none", 1.0, 0.0)
    for x, y in zip(fz, fromm):
        assert torch.allclose(x, y, rtol=0, atol=1e-15)


CASES = {
    "channel": lambda: synth.subsonic_channel(40, 16, seed=2),
    "ramp": lambda: synth.compression_ramp(40, 28),
    "box": lambda: synth.characteristic_box_3d((12, 10, 8), seed=1),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_freeze_keeps_residual_then_holds(name):
    case = CASES[name]()
    P = Problem(case)
    Q = P.initial_state()
    R0 = torch.cat([r.reshape(case.nvar, -1) for r in P.residual(Q)], 1)
    P.freeze_limiter(Q)
    R1 = torch.cat([r.reshape(case.nvar, -1) for r in P.residual(Q)], 1)
    scale = R0.abs().amax(1, keepdim=True)
    assert float(((R1 - R0).abs() / scale).max()) < 1e-13
    # two steps later the frozen residual is not the live one, and the
    # factors did not move
    phi0 = [[f.clone() for f in b] for b in P.frozen]
    for _ in range(2):
        Q, _dt = P.rk_step(Q)
    Rf = torch.cat([r.reshape(case.nvar, -1) for r in P.residual(Q)], 1)
    assert all(torch.equal(x, y) for bx, by in zip(phi0, P.frozen) for x, y in zip(bx, by))
    P.unfreeze_limiter()
    Rl = torch.cat([r.reshape(case.nvar, -1) for r in P.residual(Q)], 1)
    assert float(((Rf - Rl).abs() / scale).max()) > 1e-8


def test_freeze_rejects_no_limiter():
    case = synth.gaussian_bump_periodic(16, 16, limiter="none")
    P = Problem(case)
    with pytest.raises(ValueError):
        P.freeze_limiter(P.initial_state())
