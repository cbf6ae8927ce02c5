"""GPU tests of the debug checks (cfd_config.debug_flags).

* CFD_NAN_GHOSTS: every ghost fill first writes NaN into the whole ghost
  region (both layers, edges, corners).  Every case must give results bit for
  bit equal to the run without the flag: the connections and patches fill
  every ghost value the kernels use, and no NaN from an unfilled corner
  reaches a result.
* CFD_CHECK_FINITE: a run that goes non-physical (a fixed step far beyond the
  stability limit) stops with CFD_ERR_NONFINITE naming the step; a healthy run
  passes and is bit for bit equal to the unchecked one.
"""
import sys

import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _solver(case, **kw):
    from paper_2012_02925_amd.solver import Solver
    return Solver.from_case(case, device="cuda:0", **kw)


def _viscous(case, mu, noslip=False):
    case.scheme.viscosity = mu
    if noslip:
        for p in case.bcs:
            if p.kind == synth.SLIP_WALL:
                p.kind = synth.NOSLIP_WALL
    case.name += "_ns"
    return case


CASES = {
    "bump_64": lambda: synth.gaussian_bump_periodic(64, 64, seed=0),
    "bump_thin_2x37": lambda: synth.gaussian_bump_periodic(2, 37, seed=13),
    "ramp_100x70": lambda: synth.compression_ramp(100, 70),
    "box3d_40x36x34": lambda: synth.jittered_periodic_box(dims=(40, 36, 34), seed=4),
    "box3d_thin_3x2x5": lambda: synth.jittered_periodic_box(dims=(3, 2, 5), seed=12),
    "patchwork_small": lambda: synth.patchwork(seed=1, side_lo=16, side_hi=48),
    "subsonic_channel": lambda: synth.subsonic_channel(96, 32, seed=2),
    "farfield_bump": lambda: synth.farfield_bump(96, 48, seed=3),
    "char_box3d": lambda: synth.characteristic_box_3d((40, 36, 34), seed=10),
    "ns_square": lambda: _viscous(synth.jittered_periodic_square(48, 40, seed=3), 0.01),
    "ns_ramp_noslip": lambda: _viscous(synth.compression_ramp(100, 70), 1e-3, noslip=True),
    "ns_char_box3d_noslip": lambda: _viscous(synth.characteristic_box_3d((40, 36, 34), seed=10), 5e-3, noslip=True),
    # periodic along every axis: the viscous pass reads those neighbours through the wrap
    "ns_box3d_periodic": lambda: _viscous(synth.jittered_periodic_box(dims=(40, 36, 34), seed=4), 5e-3),
}


def _residual_and_steps(case, flags, steps=5):
    s = _solver(case, debug_flags=flags)
    out = []
    for v in range(s.query("nvariants")):
        s.set_variant(v)
        out.append(s.residual().cpu())
    s.set_variant(0)
    s.rk_step(steps)
    out.append(s.get_state().cpu())
    pads = [p.cpu() for p in s.padded_primitives()]
    s.close()
    return out, pads


@pytest.mark.parametrize("name", sorted(CASES))
def test_nan_ghosts_bitwise(name):
    from paper_2012_02925_amd import capi
    _say("case:", name, "with NaN ghosts and finite checks")
    case = CASES[name]()
    ref, _ = _residual_and_steps(case, 0)
    got, pads = _residual_and_steps(case, capi.NAN_GHOSTS | capi.CHECK_FINITE)
    for a, b in zip(ref, got):
        assert torch.equal(a, b), name
    # the ghost region really held NaN: the corner ghosts are never filled
    p = pads[0]
    corner = p[..., 0, 0] if case.dim == 2 else p[..., 2, 0, 0]
    assert torch.isnan(corner).all(), name


def test_nan_ghosts_residual_vjp_bitwise():
    """The residual VJP (2D tile pass, boundary transposes) reads only filled
    ghost values too."""
    from paper_2012_02925_amd import capi
    eps = 1e-2
    case = synth.compression_ramp(96, 64, limiter="vanalbada", lim_eps=[eps, eps, eps, eps / 1.4])
    outs = []
    for flags in (0, capi.NAN_GHOSTS):
        s = _solver(case, adjoint=True, debug_flags=flags)
        Rb = torch.randn((s.nvar, s.ncells), dtype=torch.float64, generator=torch.Generator().manual_seed(3))
        Qb, Xb, Tb = s.residual_vjp(Rb.to("cuda:0"), nodes=True, inflow=True)
        outs.append([Qb.cpu(), Xb.cpu(), Tb.cpu()])
        s.close()
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_check_finite_stops_a_blown_up_run():
    from paper_2012_02925_amd import capi
    case = synth.gaussian_bump_periodic(32, 32, seed=0, amp=0.3)
    case.scheme.dt_fixed = 5.0  # about 400 times the CFL step: the state goes non-physical
    s = _solver(case, debug_flags=capi.CHECK_FINITE)
    with pytest.raises(capi.CfdError) as exc:
        s.rk_step(50)
    assert exc.value.status == -6, exc.value
    assert "step" in str(exc.value)
    _say("  reported:", exc.value)
    s.close()


def test_check_finite_healthy_run_bitwise():
    from paper_2012_02925_amd import capi
    case = synth.compression_ramp(100, 70)
    outs = []
    for flags in (0, capi.CHECK_FINITE):
        s = _solver(case, debug_flags=flags)
        s.rk_step(10)
        outs.append(s.get_state().cpu())
        s.close()
    assert torch.equal(outs[0], outs[1])
