"""Pins for the oracle's characteristic boundary states (farfield, subsonic
inflow, subsonic outflow) and the farfield flux override, no GPU.

The states are checked against the conditions that define them, evaluated
here from the returned state: the outgoing and incoming Riemann invariants,
entropy and tangential velocity of the upwind side, the supersonic limits,
the stagnation state of the subsonic inflow, the back pressure of the outflow;
and the solver against free-stream preservation on curvilinear grids closed by
these boundaries."""
import numpy as np
import pytest
import torch

import synth
from oracle import Problem, bc

G = 1.4


def sound(q):
    return torch.sqrt(G * q[-1] / q[0])


def unit(v):
    v = torch.as_tensor(v, dtype=torch.float64)
    return v / torch.sqrt((v * v).sum())


def col(x):
    return torch.as_tensor(x, dtype=torch.float64).reshape(-1, 1)


def riemann(q, n):
    vn = (q[1:-1] * n).sum(0)
    c = sound(q)
    return vn + 2.0 * c / (G - 1.0), vn - 2.0 * c / (G - 1.0)


def entropy(q):
    return q[-1] / q[0] ** G


def tangential(q, n):
    u = q[1:-1]
    return u - (u * n).sum(0) * n


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_farfield_subsonic_invariants(dim, sign):
    """Subsonic boundary: R+ from the interior, R- from the free stream,
    entropy and tangential velocity from the upwind side."""
    rng = np.random.default_rng(11 + dim)
    n = col(unit(rng.normal(size=dim)))
    checked = 0
    for trial in range(20):
        qi = col([1.0 + 0.2 * rng.random()] + list(0.3 * rng.normal(size=dim)) + [0.7 + 0.1 * rng.random()])
        qf = col([1.0 + 0.1 * rng.random()] + list(0.3 * rng.normal(size=dim)) + [0.7 + 0.1 * rng.random()])
        # push the normal velocities to one side so both signs of V_b occur
        qi[1:-1] += sign * 0.2 * n
        qf[1:-1] += sign * 0.2 * n
        if (qf[1:-1] * n).sum().item() <= -sound(qf).item() or (qi[1:-1] * n).sum().item() >= sound(qi).item():
            continue  # supersonic: covered by the next test
        checked += 1
        qb = bc.farfield_state(qi, n, qf[:, 0], G)
        Rp_b, Rm_b = riemann(qb, n)
        Rp_i, _ = riemann(qi, n)
        _, Rm_f = riemann(qf, n)
        assert torch.allclose(Rp_b, Rp_i, rtol=0, atol=1e-13)
        assert torch.allclose(Rm_b, Rm_f, rtol=0, atol=1e-13)
        vb = (qb[1:-1] * n).sum(0)
        up = qi if vb.item() >= 0 else qf
        assert torch.allclose(entropy(qb), entropy(up), rtol=1e-13, atol=0)
        assert torch.allclose(tangential(qb, n), tangential(up, n), rtol=0, atol=1e-14)
    assert checked >= 15


def test_farfield_supersonic_limits_and_free_stream():
    n = col([0.6, 0.8])
    qf = col([1.0, 0.0, 0.0, 1.0 / G])
    # supersonic outflow: interior state kept
    qi = col([1.0, 2.0 * 0.6, 2.0 * 0.8, 1.0 / G])
    assert torch.equal(bc.farfield_state(qi, n, qf[:, 0], G), qi)
    # supersonic inflow: free stream imposed whatever the interior holds
    qfs = col([1.2, -1.9 * 0.6, -1.9 * 0.8, 0.8])
    qi2 = col([0.9, 0.1, -0.2, 0.6])
    assert torch.equal(bc.farfield_state(qi2, n, qfs[:, 0], G), qfs)
    # interior equal to the free stream: the boundary state is the free stream
    for vel in ([0.3, 0.1], [-0.3, 0.2], [0.0, 0.0]):
        q = col([1.1] + vel + [0.75])
        assert torch.allclose(bc.farfield_state(q, n, q[:, 0], G), q, rtol=1e-14, atol=1e-15)


def stagnation(q):
    c2 = G * q[-1] / q[0]
    m2 = (q[1:-1] ** 2).sum(0) / c2
    f = 1.0 + 0.5 * (G - 1.0) * m2
    return q[-1] * f ** (G / (G - 1.0)), q[0] * f ** (1.0 / (G - 1.0))


@pytest.mark.parametrize("dim", [2, 3])
def test_subsonic_inflow_stagnation_state(dim):
    rng = np.random.default_rng(5)
    d = unit(rng.normal(size=dim))
    p0, r0 = synth.stagnation_state(0.45)
    prm = torch.tensor([p0, r0] + (3.0 * d).tolist())  # unnormalised direction
    pi = torch.tensor([0.55, 0.6, 0.65, 0.7, p0 * 1.3])
    qi = torch.stack([torch.full_like(pi, 1.0)] + [torch.full_like(pi, 0.1)] * dim + [pi])
    qb = bc.subsonic_inflow_state(qi, prm, G)
    ps, rs = stagnation(qb)
    assert torch.allclose(ps, torch.full_like(ps, p0), rtol=1e-13, atol=0)
    assert torch.allclose(rs, torch.full_like(rs, r0), rtol=1e-13, atol=0)
    # static pressure from the interior, capped at p0 (then the flow is at rest)
    assert torch.allclose(qb[-1, :-1], pi[:-1], rtol=0, atol=0)
    assert qb[-1, -1].item() == p0 and torch.all(qb[1:-1, -1] == 0.0)
    # velocity along the direction
    speed = torch.sqrt((qb[1:-1] ** 2).sum(0))
    assert torch.allclose(qb[1:-1], speed * d.reshape(-1, 1), rtol=0, atol=1e-15)


def test_subsonic_outflow():
    n = col([0.0, 1.0, 0.0])
    qi = torch.tensor([[1.0, 1.0], [0.1, 0.1], [0.5, 2.0], [0.0, 0.0], [0.7, 0.7]])
    qb = bc.subsonic_outflow_state(qi, n, torch.tensor(0.65), G)
    # subsonic column: only the pressure replaced
    assert torch.equal(qb[:-1, 0], qi[:-1, 0]) and qb[-1, 0].item() == 0.65
    # supersonic column (v = 2 > c = 0.99): interior kept
    assert torch.equal(qb[:, 1], qi[:, 1])


def uniform(case, q):
    case.prims = [np.broadcast_to(np.asarray(q, float)[:, None, None] if case.dim == 2
                                  else np.asarray(q, float)[:, None, None, None],
                                  case.prims[0].shape).copy()]
    return case


@pytest.mark.parametrize("mach,alpha", [(0.6, 3.0), (1.6, 10.0), (0.3, -20.0)])
def test_farfield_box_preserves_free_stream(mach, alpha):
    """Farfield on every face of a curvilinear block: the uniform free stream
    is a steady solution (the override flux must carry the stored area
    vector with its orientation on each face)."""
    case = synth.farfield_bump(40, 24, mach=mach, alpha_deg=alpha)
    qinf = case.meta["qinf"]
    for p in case.bcs:
        p.kind, p.params = synth.FARFIELD, qinf
    uniform(case, qinf)
    P = Problem(case)
    R = P.residual(P.initial_state())[0]
    assert R.abs().max().item() < 1e-12, R.abs().max().item()
    # a perturbed free stream is not steady: the override flux differs from
    # the interior Roe flux near the boundary and the solver sees it
    q2 = np.array(qinf)
    q2[-1] *= 1.1
    for p in case.bcs:
        p.params = q2
    P2 = Problem(case)
    R2 = P2.residual(P2.initial_state())[0]
    assert R2.abs().max().item() > 1e-3


def test_farfield_3d_preserves_free_stream():
    case = synth.characteristic_box_3d((12, 10, 8), seed=3)
    qinf = case.meta["qinf"]
    for p in case.bcs:
        p.kind, p.params = synth.FARFIELD, qinf
    uniform(case, qinf)
    P = Problem(case)
    R = P.residual(P.initial_state())[0]
    assert R.abs().max().item() < 1e-12, R.abs().max().item()


def test_straight_channel_preserves_uniform_flow():
    """Subsonic inflow with the free stream's stagnation state and outflow at
    its static pressure keep a uniform flow in a straight channel steady."""
    case = synth.subsonic_channel(48, 16, mach=0.4)
    case.blocks[0].nodes = synth.bump_channel_nodes_2d(48, 16, bump=0.0, jitter=0.02, seed=4)
    uniform(case, [1.0, 0.4, 0.0, 1.0 / G])
    P = Problem(case)
    R = P.residual(P.initial_state())[0]
    assert R.abs().max().item() < 1e-12, R.abs().max().item()
    # a higher back pressure decelerates the flow at the outlet
    case.bcs[1].params = np.array([1.05 / G])
    P2 = Problem(case)
    R2 = P2.residual(P2.initial_state())[0]
    assert R2.abs().max().item() > 1e-3


def test_farfield_ghosts_hold_boundary_state():
    """Both ghost layers hold q_b; corner-adjacent tangential ranges included."""
    from oracle.ghosts import fill_ghosts
    case = synth.farfield_bump(20, 12, mach=0.6)
    P = Problem(case)
    q = [torch.tensor(case.prims[0])]
    S = [m[0] for m in P.metrics()]
    pad = fill_ghosts(P, q, S)[0]
    assert torch.equal(pad[:, 2:-2, 0], pad[:, 2:-2, 1])     # imin: both layers
    assert torch.equal(pad[:, 2:-2, -1], pad[:, 2:-2, -2])   # imax
    assert torch.equal(pad[:, -1, 2:-2], pad[:, -2, 2:-2])   # jmax
    assert torch.isfinite(pad[:, 2:-2, :2]).all()


def test_farfield_ghost_orientation_supersonic():
    """Mach 1.6 along +x (angle 10 deg): imin is a supersonic inflow (ghosts =
    free stream), imax a supersonic outflow (ghosts = adjacent interior);
    flipping the outward normal would swap the two."""
    from oracle.ghosts import fill_ghosts
    case = synth.farfield_bump(20, 12, mach=1.6, alpha_deg=10.0, amp=0.02)
    P = Problem(case)
    q = [torch.tensor(case.prims[0])]
    S = [m[0] for m in P.metrics()]
    pad = fill_ghosts(P, q, S)[0]
    qinf = torch.tensor(case.meta["qinf"]).reshape(-1, 1)
    assert torch.equal(pad[:, 2:-2, 1], qinf.expand(-1, 12))
    assert torch.equal(pad[:, 2:-2, -2], q[0][:, :, -1])
