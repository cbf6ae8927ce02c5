"""Pins for the oracle's grid metrics (no GPU)."""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import metrics


def test_cartesian_2d_exact():
    X = synth.cartesian_nodes_2d(5, 4, hx=0.25, hy=0.5)
    (Si, Sj), vol = metrics.metrics(X)
    assert torch.equal(Si[0], torch.full((4, 6), 0.5)) and torch.equal(Si[1], torch.zeros(4, 6))
    assert torch.equal(Sj[1], torch.full((5, 5), 0.25)) and torch.equal(Sj[0], torch.zeros(5, 5))
    assert torch.equal(vol, torch.full((4, 5), 0.125))


def test_cartesian_3d_exact():
    n = 4
    g = np.arange(n + 1) * 0.5
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    (Si, Sj, Sk), vol = metrics.metrics(np.stack([X, Y, Z]))
    for d, S in enumerate((Si, Sj, Sk)):
        for c in range(3):
            assert torch.equal(S[c], torch.full_like(S[c], 0.25 if c == d else 0.0))
    assert torch.equal(vol, torch.full((n, n, n), 0.125))


def _closure_2d(S, vol):
    Si, Sj = S
    return (Si[:, :, 1:] - Si[:, :, :-1]) + (Sj[:, 1:, :] - Sj[:, :-1, :])


def test_closure_and_total_area_ramp():
    ni, nj = 48, 20  # ni divisible by 3 puts a node on the ramp corner
    X = synth.ramp_nodes_2d(ni, nj)
    S, vol = metrics.metrics(X)
    assert _closure_2d(S, vol).abs().max() < 1e-16
    exact = 1.5 - 0.5 * math.tan(math.radians(10.0))  # polygon area under y = 1 above the wall
    assert abs(vol.sum().item() - exact) < 1e-14
    assert vol.min() > 0


def test_closure_and_volume_jittered_3d():
    X = synth.jittered_periodic_nodes_3d(6, 7, 5, seed=3)
    (Si, Sj, Sk), vol = metrics.metrics(X)
    clo = (Si[..., 1:] - Si[..., :-1]) + (Sj[:, :, 1:, :] - Sj[:, :, :-1, :]) + (Sk[:, 1:] - Sk[:, :-1])
    assert clo.abs().max() < 1e-16
    assert abs(vol.sum().item() - 1.0) < 1e-14
    assert vol.min() > 0


def _trilinear_volume_gauss(P):
    """Volume of the trilinear hexahedron with corner nodes P[:, k, j, i]:
    integral of det(dX/dxi) over the unit cube with 2-point Gauss rules in
    each direction (exact: det J has degree <= 2 per variable)."""
    g = [0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)]
    V = 0.0
    for u in g:
        for t in g:
            for s in g:
                # derivatives of the trilinear shape functions
                dS = np.zeros((3, 3))
                for k in range(2):
                    for j in range(2):
                        for i in range(2):
                            ws = (s if i else 1 - s)
                            wt = (t if j else 1 - t)
                            wu = (u if k else 1 - u)
                            d = np.array([(1 if i else -1) * wt * wu,
                                          ws * (1 if j else -1) * wu,
                                          ws * wt * (1 if k else -1)])
                            dS += np.outer(P[:, k, j, i], d)
                V += 0.125 * np.linalg.det(dS)
    return V


def test_hex_volume_equals_trilinear_volume():
    rng = np.random.default_rng(7)
    base = np.stack(np.meshgrid([0.0, 1.0], [0.0, 1.0], [0.0, 1.0], indexing="ij")[::-1])
    for _ in range(10):
        P = base + 0.2 * rng.standard_normal(base.shape)
        _, vol = metrics.metrics(P)
        assert vol.item() == pytest.approx(_trilinear_volume_gauss(P), rel=1e-13)


def test_quad_area_equals_bilinear_area():
    rng = np.random.default_rng(8)
    for _ in range(10):
        X = np.stack(np.meshgrid([0.0, 1.0], [0.0, 1.0], indexing="xy")) + 0.2 * rng.standard_normal((2, 2, 2))
        _, vol = metrics.metrics(X)
        x, y = X[0], X[1]
        # shoelace over the polygon (0,0) (1,0) (1,1) (0,1) in node-index terms
        px = [x[0, 0], x[0, 1], x[1, 1], x[1, 0]]
        py = [y[0, 0], y[0, 1], y[1, 1], y[1, 0]]
        area = 0.5 * sum(px[m] * py[(m + 1) % 4] - px[(m + 1) % 4] * py[m] for m in range(4))
        assert vol.item() == pytest.approx(area, rel=1e-13)
