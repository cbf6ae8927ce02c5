"""Pins for the oracle's limiters and kappa-form MUSCL face states (no GPU)."""
import numpy as np
import pytest
import torch

from oracle import muscl

LIMITERS = ["none", "vanleer", "vanalbada"]


def test_slope_equals_psi_times_denominator():
    rng = np.random.default_rng(0)
    a = torch.tensor(rng.standard_normal(500))
    b = torch.tensor(rng.standard_normal(500))
    for lim in LIMITERS:
        assert torch.allclose(muscl.slope(a, b, lim), muscl.psi(a / b, lim) * b, rtol=1e-13, atol=1e-15)


def test_textbook_limiter_values():
    r = torch.tensor([-2.0, -0.5, 0.0, 0.5, 1.0, 2.0, 10.0])
    vl = muscl.psi(r, "vanleer")
    assert torch.allclose(vl, torch.tensor([0, 0, 0, 2 / 3, 1, 4 / 3, 20 / 11.0]))
    va = muscl.psi(r, "vanalbada")
    assert torch.allclose(va, torch.tensor([2 / 5, -1 / 5, 0, 3 / 5, 1, 6 / 5, 110 / 101.0]))


@pytest.mark.parametrize("lim", LIMITERS)
def test_psi_one_and_zero_rule(lim):
    # (values below about 1e-100 underflow in the products of the slope
    # form; both the oracle and the kernels share that property)
    a = torch.tensor([0.3, -2.0, 1e-90, 0.0])
    assert torch.equal(muscl.slope(a, a, lim), a)
    if lim != "none":
        z = torch.zeros(3)
        assert torch.equal(muscl.slope(z, z, lim), z)


def test_vanleer_extrema_and_symmetry():
    rng = np.random.default_rng(1)
    a = torch.tensor(rng.standard_normal(1000))
    b = torch.tensor(rng.standard_normal(1000))
    s = muscl.slope(a, b, "vanleer")
    assert torch.all(s[(a * b) <= 0] == 0)
    for lim in ("vanleer", "vanalbada"):
        e2 = torch.full_like(a, 0.01)
        assert torch.equal(muscl.slope(a, b, lim, e2), muscl.slope(b, a, lim, e2))


def _states(q1d, lim, eps, kappa):
    q = torch.as_tensor(q1d)[None, :]
    return muscl.face_states(q, 1, lim, eps, kappa)


@pytest.mark.parametrize("lim", LIMITERS)
def test_linear_data_reconstructed_exactly(lim):
    q = torch.arange(-2, 12, dtype=torch.float64) * 0.37 + 1.1  # padded cells -2..11 of n = 10
    qL, qR = _states(q, lim, 1.0, -1.0)
    faces = (torch.arange(0, 11, dtype=torch.float64) - 0.5) * 0.37 + 1.1
    assert torch.allclose(qL[0], faces, rtol=1e-14)
    assert torch.allclose(qR[0], faces, rtol=1e-14)


@pytest.mark.parametrize("kappa,expect_offset", [(-1.0, -0.5), (1.0 / 3.0, 1.0 / 6.0), (0.0, 0.0), (1.0, 0.5)])
def test_quadratic_closed_form_unlimited(kappa, expect_offset):
    """q_i = i^2 with Psi = 1 and eps = 1: eq. (flux) evaluated by hand gives
    q^L_{i+1/2} = q^R_{i+1/2} = i^2 + i + kappa/2 (the exact point value at
    i + 1/2 is i^2 + i + 1/4)."""
    idx = torch.arange(-2, 12, dtype=torch.float64)
    qL, qR = _states(idx ** 2, "none", 1.0, kappa)
    i = torch.arange(-1, 10, dtype=torch.float64)  # left cell of faces 0..10
    assert torch.allclose(qL[0], i * i + i + expect_offset, rtol=0, atol=1e-12)
    assert torch.allclose(qR[0], i * i + i + expect_offset, rtol=0, atol=1e-12)


@pytest.mark.parametrize("lim", ["vanleer", "vanalbada"])
def test_kappa_independence_for_symmetric_limiters(lim):
    rng = np.random.default_rng(2)
    q = torch.tensor(rng.standard_normal((3, 30)))
    ref = muscl.face_states(q, 1, lim, 1.0, -1.0)
    for kappa in (0.0, 1.0 / 3.0, 0.5, 1.0):
        got = muscl.face_states(q, 1, lim, 1.0, kappa)
        assert torch.allclose(got[0], ref[0], rtol=1e-13, atol=1e-14)
        assert torch.allclose(got[1], ref[1], rtol=1e-13, atol=1e-14)


def test_vanalbada_regularised_is_smooth():
    e2 = torch.tensor(1e-4)
    rng = np.random.default_rng(3)
    for a0, b0 in [(0.0, 0.0), (1e-3, -2e-3)] + [tuple(rng.standard_normal(2) * 0.01) for _ in range(5)]:
        a = torch.tensor(a0, requires_grad=True)
        b = torch.tensor(b0, requires_grad=True)
        s = muscl.slope(a, b, "vanalbada", e2)
        ga, gb = torch.autograd.grad(s, (a, b))
        h = 1e-7
        fa = (muscl.slope(torch.tensor(a0 + h), torch.tensor(b0), "vanalbada", e2)
              - muscl.slope(torch.tensor(a0 - h), torch.tensor(b0), "vanalbada", e2)) / (2 * h)
        fb = (muscl.slope(torch.tensor(a0), torch.tensor(b0 + h), "vanalbada", e2)
              - muscl.slope(torch.tensor(a0), torch.tensor(b0 - h), "vanalbada", e2)) / (2 * h)
        assert abs(ga - fa) < 1e-7 and abs(gb - fb) < 1e-7
    a = torch.tensor(0.0, requires_grad=True)
    b = torch.tensor(0.0, requires_grad=True)
    ga, gb = torch.autograd.grad(muscl.slope(a, b, "vanalbada", e2), (a, b))
    assert ga.item() == pytest.approx(0.5) and gb.item() == pytest.approx(0.5)
