"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Every test calls the library through its C ABI (paper_2012_02925_amd.capi via
Solver) and compares element by element with tolerances from parity_util.
"""
import copy
import sys

import numpy as np
import pytest
import torch

import synth
from parity_util import (compare_residual, compare_state, ghost_mask, oracle_padded, oracle_residual, oracle_run,
                         q_ref, residual_scale)

pytestmark = pytest.mark.gpu


def _solver(case, **kw):
    from paper_2012_02925_amd.solver import Solver
    return Solver.from_case(case, device="cuda:0", **kw)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_residual(case, variants=None):
    s = _solver(case)
    P, Q0, Rref = oracle_residual(case)
    qr = q_ref(case)
    rs = residual_scale(case, qr)
    nvar = s.query("nvariants")
    for v in (range(nvar) if variants is None else variants):
        s.set_variant(v)
        R = s.residual()
        torch.cuda.synchronize()
        ok, rep = compare_residual(R, Rref, qr, rs)
        _say("  variant", v, rep)
        assert ok, (case.name, "variant", v, rep)
    return s


def test_library_loads_on_gpu():
    from paper_2012_02925_amd import capi
    assert torch.cuda.is_available()
    capi.load()


@pytest.mark.parametrize("lim", ["vanleer", "vanalbada", "none"])
def test_bump_residual_all_variants(lim):
    _say("case: gaussian bump 64x64", lim)
    check_residual(synth.gaussian_bump_periodic(64, 64, seed=0, limiter=lim))


def test_bump_ghost_fill():
    case = synth.gaussian_bump_periodic(64, 64, seed=1)
    s = _solver(case)
    pad = s.padded_primitives()
    ref = oracle_padded(case)
    m = ghost_mask(2, pad[0].shape)
    d = (pad[0].cpu() - ref[0]).abs()[:, m]
    assert d.max() <= 1e-15, d.max()


def test_bump_time_step_and_100_steps():
    _say("case: gaussian bump 64x64, 100 steps")
    case = synth.gaussian_bump_periodic(64, 64, seed=0)
    s = _solver(case)
    dt0 = s.time_step().item()
    Qref, dts = oracle_run(case, 100)
    assert abs(dt0 - dts[0]) <= 1e-14 * dts[0], (dt0, dts[0])
    dt_last = torch.empty(1, dtype=torch.float64, device="cuda:0")
    s.rk_step(100, dt_last)
    Q = s.get_state()
    torch.cuda.synchronize()
    assert abs(dt_last.item() - dts[-1]) <= 1e-12 * dts[-1]
    ok, rep = compare_state(Q, Qref, q_ref(case))
    assert ok, rep


def test_ramp_reduced_residual_and_steps():
    _say("case: ramp 100x70")
    case = synth.compression_ramp(100, 70)
    s = check_residual(case)
    s.set_variant(0)
    Qref, dts = oracle_run(case, 30)
    s.rk_step(30)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    assert ok, rep


def test_box3d_reduced_residual_and_steps():
    _say("case: jittered box 40x36x34")
    case = synth.jittered_periodic_box(dims=(40, 36, 34), seed=4)
    s = check_residual(case)
    Qref, dts = oracle_run(case, 4)
    s.rk_step(4)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    assert ok, rep


@pytest.mark.parametrize("dims", [(2, 9, 2), (3, 2, 5), (37, 3, 2), (2, 2, 2), (2, 37, 1), (45, 3, 1)])
def test_thin_blocks_residual_and_steps(dims):
    """Blocks two or three cells thin: most lanes of a tile lie outside the
    padded block, where the stage kernel's loads take clamped in-bounds
    addresses and the results are discarded; every tile variant's residual and
    four RK steps against the oracle."""
    _say("case: thin periodic block", dims)
    case = (synth.gaussian_bump_periodic(dims[0], dims[1], seed=13) if dims[2] == 1
            else synth.jittered_periodic_box(dims=dims, seed=12))
    s = check_residual(case)
    Qref, dts = oracle_run(case, 4)
    s.rk_step(4)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    assert ok, rep


FVS = ["vanleer_fvs", "steger_warming"]


def _with_flux(case, flux):
    case.scheme.flux = flux
    case.name = case.name + "_" + flux
    return case


@pytest.mark.parametrize("flux", FVS)
@pytest.mark.parametrize("lim", ["vanleer", "none"])
def test_fvs_bump_residual_all_variants_and_steps(flux, lim):
    _say("case: gaussian bump 64x64", flux, lim)
    case = _with_flux(synth.gaussian_bump_periodic(64, 64, seed=2, limiter=lim), flux)
    s = check_residual(case)
    Qref, dts = oracle_run(case, 20)
    s.rk_step(20)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    assert ok, rep


@pytest.mark.parametrize("flux", FVS)
def test_fvs_ramp_reduced_residual_and_steps(flux):
    """Mach 2.5 inflow (van Leer's supersonic branches), subsonic pockets
    behind the shock and slip-wall faces."""
    _say("case: ramp 100x70", flux)
    case = _with_flux(synth.compression_ramp(100, 70), flux)
    s = check_residual(case)
    s.set_variant(1)
    Qref, dts = oracle_run(case, 30)
    s.rk_step(30)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    assert ok, rep


@pytest.mark.parametrize("flux", FVS)
def test_fvs_box3d_reduced_residual_and_steps(flux):
    _say("case: jittered box 40x36x34", flux)
    case = _with_flux(synth.jittered_periodic_box(dims=(40, 36, 34), seed=6), flux)
    s = check_residual(case)
    Qref, dts = oracle_run(case, 4)
    s.rk_step(4)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    assert ok, rep


def test_box3d_ghost_fill():
    case = synth.jittered_periodic_box(dims=(20, 18, 17), seed=5)
    s = _solver(case)
    pad = s.padded_primitives()
    ref = oracle_padded(case)
    m = ghost_mask(3, pad[0].shape)
    d = (pad[0].cpu() - ref[0]).abs()[:, m]
    assert d.max() <= 1e-15, d.max()


@pytest.mark.parametrize("mode,graph", [("batched", True), ("batched", False), ("per_block", False),
                                        ("persistent", True), ("persistent", False)])
def test_patchwork_small_modes(mode, graph):
    _say("case: patchwork 3x3", mode, graph)
    case = synth.patchwork(seed=2, nbx=3, nby=3, side_lo=8, side_hi=40, h=1.0 / 64)
    s = _solver(case)
    s.set_exec(mode, graph)
    P, Q0, Rref = oracle_residual(case)
    qr = q_ref(case)
    ok, rep = compare_residual(s.residual(), Rref, qr, residual_scale(case, qr))
    assert ok, rep
    Qref, _ = oracle_run(case, 12)
    s.rk_step(12)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    assert ok, rep


def test_modes_are_bitwise_identical():
    """Every execution mode (batched, persistent, per block; with and without
    the captured step graph) and both ghost exchanges (direct copy, packed)
    give the same bits."""
    case = synth.patchwork(seed=3, nbx=3, nby=2, side_lo=10, side_hi=50, h=1.0 / 64)
    outs = []
    for mode, graph, ghosts in [("batched", True, "direct"), ("batched", False, "direct"),
                                ("per_block", False, "direct"), ("persistent", True, "direct"),
                                ("persistent", False, "direct"), ("batched", True, "packed"),
                                ("per_block", False, "packed"), ("persistent", True, "packed")]:
        s = _solver(case)
        s.set_exec(mode, graph)
        s.set_ghost_exchange(ghosts)
        s.rk_step(7)
        outs.append((mode, graph, ghosts, s.get_state().cpu()))
        s.close()
    for o in outs[1:]:
        assert torch.equal(outs[0][3], o[3]), o[:3]


@pytest.mark.parametrize("ghosts", ["direct", "packed"])
def test_ghost_exchange_modes_3d_oriented(ghosts):
    """Both exchanges on the 3D two-block box whose connections swap and
    reverse tangential axes: ghost fill against the oracle at 1e-15 and the
    persistent launch's residual against the oracle."""
    case = _rotated_two_block_box()
    s = _solver(case)
    s.set_ghost_exchange(ghosts)
    s.set_exec("persistent", True)
    pad = s.padded_primitives()
    ref = oracle_padded(case)
    for b in range(2):
        m = ghost_mask(3, pad[b].shape)
        d = (pad[b].cpu() - ref[b]).abs()[:, m]
        assert d.max() <= 1e-15, (b, float(d.max()))
    P, Q0, Rref = oracle_residual(case)
    qr = q_ref(case)
    ok, rep = compare_residual(s.residual(), Rref, qr, residual_scale(case, qr))
    assert ok, rep


@pytest.mark.parametrize("dims", [(33, 21, 40), (40, 36, 34), (32, 32, 32)])
def test_variants_are_bitwise_identical_3d(dims):
    """Every tile variant gives the same bits, for the residual and over 3
    steps.  The extents make the block's high boundary faces fall on tile
    edges in some variants and on ghost-cell lanes in others."""
    case = synth.jittered_periodic_box(dims=dims, seed=6)
    ni, nj = dims[0], dims[1]
    s = _solver(case)
    outs, states = [], []
    for v in range(s.query("nvariants")):
        s.set_variant(v)
        outs.append(s.residual().cpu())
    s.close()
    for v in range(len(outs)):
        s = _solver(case)
        s.set_variant(v)
        s.rk_step(3)
        states.append(s.get_state().cpu())
        s.close()
    for v, o in enumerate(outs[1:], 1):
        d = (o - outs[0]).abs()
        if d.max() > 0:
            flat = int(d.max(dim=0).values.argmax())
            _say("variant", v, "max diff", float(d.max()), "at cell (i,j,k) =",
                 (flat % ni, (flat // ni) % nj, flat // (ni * nj)), "count", int((d > 0).sum()))
        assert torch.equal(o, outs[0])
        assert torch.equal(states[v], states[0]), v


def _sheared_periodic_box(dims=(24, 20, 18), seed=2):
    """The jittered box connected to itself along every axis, but sheared
    (x += 0.1 y^2, y += 0.1 z^2, z += 0.1 x^2) so that the faces at the two
    ends of each axis differ in shape: the connections pair cells whose
    boundary faces are not translates of each other."""
    case = synth.jittered_periodic_box(dims=dims, seed=seed)
    X = case.blocks[0].nodes
    x, y, z = X[0].copy(), X[1].copy(), X[2].copy()
    X[0] = x + 0.1 * y * y
    X[1] = y + 0.1 * z * z
    X[2] = z + 0.1 * x * x
    case.name += "_sheared"
    return case


def test_sheared_periodic_box_residual_and_steps():
    """Periodic neighbours are read through the wrap but every face keeps its
    own area vector: residual (all tile variants) and 10 steps against the
    oracle on a box whose opposite ends have different face geometry."""
    case = _sheared_periodic_box()
    check_residual(case)
    Qref, dref = oracle_run(case, 10)
    for v in (0, 2):
        s = _solver(case)
        s.set_variant(v)
        dt = torch.empty(1, dtype=torch.float64, device="cuda:0")
        dts = []
        for _ in range(10):
            s.rk_step(1, dt)
            dts.append(dt.item())
        ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
        _say("  variant", v, rep)
        assert ok, rep
        assert max(abs(a - b) / b for a, b in zip(dts, dref)) <= 1e-12
        s.close()


def test_local_time_stepping_ramp():
    """Local time stepping (every cell with its own CFL step from Q^n) on the
    reduced ramp: state after 25 steps and the reported smallest step."""
    _say("case: ramp 100x70, local time stepping, 25 steps")
    case = synth.compression_ramp(100, 70)
    case.scheme.local_dt = True
    s = _solver(case)
    Qref, dts = oracle_run(case, 25)
    dt_last = torch.empty(1, dtype=torch.float64, device="cuda:0")
    s.rk_step(25, dt_last)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    assert ok, rep
    assert abs(dt_last.item() - dts[-1]) <= 1e-12 * dts[-1]


@pytest.mark.parametrize("dims", [(64, 64, 1), (40, 36, 34)])
def test_residual_norms(dims):
    import oracle
    case = (synth.gaussian_bump_periodic(dims[0], dims[1], seed=5) if dims[2] == 1
            else synth.jittered_periodic_box(dims=dims, seed=7))
    s = _solver(case)
    R, N = s.residual_norms()
    P = oracle.Problem(case)
    Nref = P.residual_norms(P.initial_state())
    # components whose residual is rounding-level (the bump's y-momentum)
    # are bounded like the residual itself: 1e-12 of the reference flux scale
    err = (N.cpu() - Nref).abs()
    bound = 1e-11 * Nref + 1e-12 * torch.as_tensor(residual_scale(case, q_ref(case)), dtype=torch.float64)
    _say("  norms", N.cpu().tolist(), "err", err.tolist())
    assert (err <= bound).all(), (err, bound)


# characteristic boundaries: farfield (Riemann invariants, exact-flux face
# override), subsonic inflow from stagnation conditions, back-pressure outflow
CHAR_CASES = {
    # ragged tiles in both directions; subsonic farfield on imin, imax, jmax
    "farfield_M0.6_100x70": lambda: synth.farfield_bump(100, 70, mach=0.6, alpha_deg=3.0, seed=1),
    # supersonic inflow and outflow branches, subsonic normal flow on jmax
    "farfield_M1.6_96x48": lambda: synth.farfield_bump(96, 48, mach=1.6, alpha_deg=10.0, seed=2),
    # interior pressure above p0 on part of the inlet (the cap p_b = p0)
    "subsonic_channel_96x40": lambda: synth.subsonic_channel(96, 40, mach=0.5, pressure_amp=0.4, seed=5),
}


@pytest.mark.parametrize("name", sorted(CHAR_CASES))
def test_characteristic_bc_residual_and_steps(name):
    _say("case:", name)
    case = CHAR_CASES[name]()
    s = check_residual(case)
    s.set_variant(1)
    Qref, dts = oracle_run(case, 20)
    s.rk_step(20)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    assert ok, rep


def _ghost_parity(case, tol=1e-14):
    s = _solver(case)
    pad = s.padded_primitives()
    ref = oracle_padded(case)
    m = ghost_mask(case.dim, pad[0].shape)
    d = (pad[0].cpu() - ref[0]).abs()[:, m]
    # per-variable scale; the velocity components share the largest speed
    # (a farfield ghost velocity comes out of invariants of size |V| + c)
    scale = ref[0].abs()[:, m].amax(dim=1, keepdim=True)
    scale[1:-1] = scale[1:-1].max()
    _say("  ghost max rel diff", float((d / scale).max()))
    assert (d <= tol * scale).all(), float((d / scale).max())


@pytest.mark.parametrize("name", sorted(CHAR_CASES))
def test_characteristic_bc_ghost_fill(name):
    _ghost_parity(CHAR_CASES[name]())


def test_characteristic_box3d_ghosts_residual_and_steps():
    """Every characteristic kind in 3D: subsonic inflow (tilted direction) on
    imin, subsonic outflow on imax, farfield on jmax and kmin (the k-face
    override of the register queue), slip wall, extrapolation."""
    _say("case: characteristic box 40x36x34")
    case = synth.characteristic_box_3d((40, 36, 34), seed=5)
    _ghost_parity(case)
    s = check_residual(case)
    Qref, dts = oracle_run(case, 4)
    s.rk_step(4)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    assert ok, rep


@pytest.mark.parametrize("flux", FVS)
def test_fvs_farfield_residual_and_steps(flux):
    """The farfield override with the flux-vector splittings (F(q_b, q_b))."""
    _say("case: farfield M0.6 100x70", flux)
    case = _with_flux(synth.farfield_bump(100, 70, mach=0.6, seed=4), flux)
    s = check_residual(case)
    Qref, dts = oracle_run(case, 10)
    s.rk_step(10)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    assert ok, rep


def test_farfield_and_outflow_parameter_update():
    """cfd_set_bc_params on a farfield and a subsonic-outflow patch."""
    case = synth.farfield_bump(64, 40, mach=0.6, seed=6)
    s = _solver(case)
    qinf2 = np.array(case.meta["qinf"]) * np.array([1.02, 0.97, 1.0, 1.03])
    for pid, p in zip(s.patch_ids, case.bcs):
        if p.kind == synth.FARFIELD:
            s.set_bc_params(pid, qinf2)
            p.params = qinf2
    P, Q0, Rref = oracle_residual(case)
    qr = q_ref(case)
    ok, rep = compare_residual(s.residual(), Rref, qr, residual_scale(case, qr))
    assert ok, rep
    case2 = synth.subsonic_channel(64, 24, mach=0.5, seed=7)
    s2 = _solver(case2)
    s2.set_bc_params(s2.patch_ids[1], [1.1 / synth.GAMMA])
    case2.bcs[1].params = np.array([1.1 / synth.GAMMA])
    P, Q0, Rref = oracle_residual(case2)
    qr = q_ref(case2)
    ok, rep = compare_residual(s2.residual(), Rref, qr, residual_scale(case2, qr))
    assert ok, rep


# limiter freezing: live steps, freeze, frozen steps, unfreeze
FREEZE_CASES = {
    # steady machinery together: local time stepping, subsonic in/outflow
    "channel_local_dt_96x40": lambda: synth.subsonic_channel(96, 40, mach=0.5, pressure_amp=0.1, seed=5),
    # van Albada with regularisation, supersonic inflow, slip wall
    "ramp_vanalbada_100x70": lambda: synth.compression_ramp(100, 70, limiter="vanalbada",
                                                            lim_eps=[1e-2, 1e-2, 1e-2, 1e-2 / 1.4]),
    "char_box_40x36x34": lambda: synth.characteristic_box_3d((40, 36, 34), seed=8),
}


@pytest.mark.parametrize("name", sorted(FREEZE_CASES))
def test_limiter_freezing(name):
    import oracle
    _say("case:", name)
    case = FREEZE_CASES[name]()
    if name.startswith("channel"):
        case.scheme.local_dt = True
    s = _solver(case, freezing=True)
    P = oracle.Problem(case)
    met = P.metrics()
    Q = P.initial_state()
    qr = q_ref(case)
    rs = residual_scale(case, qr)
    nlive, nfrozen = (6, 10) if case.dim == 2 else (2, 3)
    for _ in range(nlive):
        Q, _dt = P.rk_step(Q, met)
    s.rk_step(nlive)
    P.freeze_limiter(Q, met)
    s.freeze_limiter(True)
    Rref = torch.cat([r.reshape(case.nvar, -1) for r in P.residual(Q, met)], 1)
    for v in range(s.query("nvariants")):
        s.set_variant(v)
        ok, rep = compare_residual(s.residual(), Rref, qr, rs)
        _say("  frozen residual, variant", v, rep)
        assert ok, rep
    s.set_variant(1)
    for _ in range(nfrozen):
        Q, _dt = P.rk_step(Q, met)
    s.rk_step(nfrozen)
    Qref = torch.cat([x.reshape(case.nvar, -1) for x in Q], 1)
    ok, rep = compare_state(s.get_state(), Qref, qr)
    _say("  after frozen steps", rep)
    assert ok, rep
    # back to the live limiter, at the oracle's state (after 16 steps the two
    # states differ by about 1e-12, which the residual next to the shock
    # amplifies beyond the single-residual bar)
    P.unfreeze_limiter()
    s.freeze_limiter(False)
    s.set_state(Qref.to("cuda:0"))
    Rref = torch.cat([r.reshape(case.nvar, -1) for r in P.residual(Q, met)], 1)
    ok, rep = compare_residual(s.residual(), Rref, qr, rs)
    assert ok, rep


def test_limiter_freezing_modes_bitwise():
    """Frozen steps are identical in the three execution modes."""
    case = synth.patchwork(seed=4, nbx=3, nby=2, side_lo=10, side_hi=40, h=1.0 / 64)
    outs = []
    for mode, graph in [("batched", True), ("batched", False), ("per_block", False)]:
        s = _solver(case, freezing=True)
        s.set_exec(mode, graph)
        s.rk_step(3)
        s.freeze_limiter(True)
        s.rk_step(4)
        outs.append(s.get_state().cpu())
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


# laminar Navier-Stokes: viscous residual (Green's-theorem face gradients),
# no-slip walls, viscous time-step term
def _viscous(case, mu, noslip=False):
    case.scheme.viscosity = mu
    if noslip:
        for p in case.bcs:
            if p.kind == synth.SLIP_WALL:
                p.kind = synth.NOSLIP_WALL
    case.name += "_ns"
    return case


NS_CASES = {
    "square_periodic_48x40": lambda: _viscous(synth.jittered_periodic_square(48, 40, seed=3), 0.01),
    "channel_noslip_96x40": lambda: _viscous(synth.subsonic_channel(96, 40, mach=0.5, seed=5), 2e-3, noslip=True),
    "ramp_noslip_100x70": lambda: _viscous(synth.compression_ramp(100, 70), 1e-3, noslip=True),
    "patchwork_3x3": lambda: _viscous(synth.patchwork(seed=2, nbx=3, nby=3, side_lo=8, side_hi=40, h=1.0 / 64), 5e-3),
}


@pytest.mark.parametrize("name", sorted(NS_CASES))
def test_navier_stokes_residual_and_steps(name):
    import oracle
    _say("case: NS", name)
    case = NS_CASES[name]()
    s = check_residual(case)
    P = oracle.Problem(case)
    dt0 = s.time_step().item()
    ref = float(P.time_step(P.initial_state()))
    assert abs(dt0 - ref) <= 1e-13 * ref, (dt0, ref)
    s.set_variant(1)
    Qref, dts = oracle_run(case, 15)
    s.rk_step(15)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    _say("  after 15 steps", rep)
    assert ok, rep


@pytest.mark.parametrize("dims", [(2, 9, 3), (3, 2, 2), (2, 17, 1), (17, 3, 1)])
def test_navier_stokes_thin_blocks(dims):
    """Laminar Navier-Stokes on periodic blocks two or three cells thin: the
    viscous pass's tiles are mostly outside the block and its pseudo-nodes
    average cells across the periodic seam on both sides; residual and four
    RK steps against the oracle."""
    _say("case: NS thin periodic block", dims)
    base = (synth.jittered_periodic_square(dims[0], dims[1], seed=15) if dims[2] == 1
            else synth.jittered_periodic_box(dims=dims, seed=14))
    case = _viscous(base, 0.01)
    s = check_residual(case)
    Qref, dts = oracle_run(case, 4)
    s.rk_step(4)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    _say("  after 4 steps", rep)
    assert ok, rep


@pytest.mark.parametrize("which", ["periodic_box", "char_box_noslip"])
def test_navier_stokes_3d(which):
    _say("case: NS 3D", which)
    if which == "periodic_box":
        case = _viscous(synth.jittered_periodic_box(dims=(40, 36, 34), seed=9), 0.01)
    else:
        case = _viscous(synth.characteristic_box_3d((40, 36, 34), seed=10), 5e-3, noslip=True)
    s = check_residual(case)
    Qref, dts = oracle_run(case, 3)
    s.rk_step(3)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    assert ok, rep


def _rotated_two_block_box(ni=20, nj=12, nk=10, cut=8, seed=9):
    """The jittered periodic box cut at i = cut; the second block rotated
    about the i axis (j' = k, k' = nj-1-j) and joined with orient 6 / 5, so
    connections swap and reverse tangential axes."""
    c = synth.jittered_periodic_box(dims=(ni, nj, nk), seed=seed)
    X, q = c.blocks[0].nodes, c.prims[0]
    XA, qA = X[:, :, :, :cut + 1].copy(), q[:, :, :, :cut].copy()
    XB, qB = X[:, :, :, cut:], q[:, :, :, cut:]
    XBr = XB.transpose(0, 2, 1, 3)[:, ::-1].copy()
    qBr = qB.transpose(0, 2, 1, 3)[:, ::-1].copy()
    nB = ni - cut
    A = synth.Block(cut, nj, nk, XA)
    B = synth.Block(nB, nk, nj, XBr)
    conns = [synth.Connection(0, synth.IMAX, [0, 0], [nj, nk], 1, synth.IMIN, [0, 0], [nk, nj], 6),
             synth.Connection(1, synth.IMAX, [0, 0], [nk, nj], 0, synth.IMIN, [0, 0], [nj, nk], 5),
             synth.Connection(0, synth.JMIN, [0, 0], [cut, nk], 0, synth.JMAX, [0, 0], [cut, nk], 0),
             synth.Connection(0, synth.KMIN, [0, 0], [cut, nj], 0, synth.KMAX, [0, 0], [cut, nj], 0),
             synth.Connection(1, synth.JMIN, [0, 0], [nB, nj], 1, synth.JMAX, [0, 0], [nB, nj], 0),
             synth.Connection(1, synth.KMIN, [0, 0], [nB, nk], 1, synth.KMAX, [0, 0], [nB, nk], 0)]
    return synth.Case("rotated_two_block_box_%dx%dx%d" % (ni, nj, nk), 3, [A, B], [], conns, [qA, qBr],
                      c.scheme, 1)


@pytest.mark.parametrize("viscous", [False, True])
def test_rotated_two_block_box_3d(viscous):
    """Oriented 3D connections (axis swap and reversal): ghost exchange and,
    with viscosity, the ghost cell centres and pseudo-nodes at block edges."""
    _say("case: rotated two-block box, viscous", viscous)
    case = _rotated_two_block_box()
    if viscous:
        case = _viscous(case, 0.01)
    s = check_residual(case)
    s.set_variant(1)
    Qref, dts = oracle_run(case, 4)
    s.rk_step(4)
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    assert ok, rep


def test_navier_stokes_modes_bitwise():
    """The viscous pass gives identical steps in the three execution modes."""
    case = _viscous(synth.patchwork(seed=5, nbx=3, nby=2, side_lo=10, side_hi=40, h=1.0 / 64), 5e-3)
    outs = []
    for mode, graph in [("batched", True), ("batched", False), ("per_block", False)]:
        s = _solver(case)
        s.set_exec(mode, graph)
        s.rk_step(5)
        outs.append(s.get_state().cpu())
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_navier_stokes_steady_machinery():
    """Viscous channel with no-slip walls, local time stepping, residual norms
    and limiter freezing together: state and norms against the oracle."""
    import oracle
    case = _viscous(synth.subsonic_channel(64, 32, mach=0.5, seed=11), 2e-3, noslip=True)
    case.scheme.local_dt = True
    s = _solver(case, freezing=True)
    P = oracle.Problem(case)
    met = P.metrics()
    Q = P.initial_state()
    for _ in range(5):
        Q, _dt = P.rk_step(Q, met)
    s.rk_step(5)
    P.freeze_limiter(Q, met)
    s.freeze_limiter(True)
    for _ in range(5):
        Q, _dt = P.rk_step(Q, met)
    s.rk_step(5)
    qr = q_ref(case)
    Qref = torch.cat([x.reshape(case.nvar, -1) for x in Q], 1)
    ok, rep = compare_state(s.get_state(), Qref, qr)
    assert ok, rep
    R, N = s.residual_norms()
    Nref = P.residual_norms(Q)
    rs = torch.as_tensor(residual_scale(case, qr), dtype=torch.float64)
    err = (N.cpu() - Nref).abs()
    assert (err <= 1e-10 * Nref + 1e-11 * rs).all(), (err, Nref)


@pytest.mark.parametrize("stages", [1, 2, 3])
def test_rk_stage_counts_match_oracle(stages):
    """M-stage schemes other than the classical four (Sec. 2): the state and
    the time steps of 12 steps against the oracle; M = 1 never updates in
    place (its stage writes a second buffer that is copied back)."""
    case = synth.jittered_periodic_box(dims=(20, 18, 16), seed=3)
    case.scheme.rk_stages = stages
    case.scheme.cfl = 0.4
    Qref, dref = oracle_run(case, 12)
    s = _solver(case)
    dt = torch.empty(1, dtype=torch.float64, device="cuda:0")
    dts = []
    for _ in range(12):
        s.rk_step(1, dt)
        dts.append(dt.item())
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    _say("  stages", stages, rep)
    assert ok, rep
    assert max(abs(a - b) / b for a, b in zip(dts, dref)) <= 1e-12


def test_periodic_wrap_with_filled_connections_all_modes():
    """The two-block box whose blocks are periodic onto themselves along j and
    k (read through the wrap by the stage kernel, not filled between stages)
    and joined to each other along i with swapped and reversed axes (filled):
    10 steps in every launch mode and both exchanges, with and without
    NaN-filled ghost regions, bit for bit equal, and within the state bar of
    the oracle."""
    from paper_2012_02925_amd import capi
    case = _rotated_two_block_box()
    outs = []
    for mode, graph, ghosts, flags in [("batched", True, "direct", 0), ("per_block", False, "direct", 0),
                                       ("persistent", True, "direct", 0), ("batched", False, "packed", 0),
                                       ("batched", False, "direct", capi.NAN_GHOSTS),
                                       ("per_block", False, "direct", capi.NAN_GHOSTS)]:
        s = _solver(case, debug_flags=flags)
        s.set_exec(mode, graph)
        s.set_ghost_exchange(ghosts)
        s.rk_step(10)
        outs.append(((mode, graph, ghosts, flags), s.get_state().cpu()))
        s.close()
    for key, o in outs[1:]:
        assert torch.equal(outs[0][1], o), key
    Qref, _ = oracle_run(case, 10)
    ok, rep = compare_state(outs[0][1], Qref, q_ref(case))
    _say("  ", rep)
    assert ok, rep


def test_autotune_picks_a_variant_and_keeps_the_bits():
    """cfd_autotune times every tile variant on the current state and keeps
    the fastest: the chosen index is valid and selected, and the run after it
    is bit for bit the run with any fixed variant."""
    case = synth.jittered_periodic_box(dims=(40, 36, 34), seed=4)
    s = _solver(case)
    v = s.autotune(3)
    assert 0 <= v < s.query("nvariants") and s.query("variant") == v
    s.rk_step(3)
    Q1 = s.get_state().cpu()
    s.close()
    s = _solver(case)
    s.set_variant(0)
    s.rk_step(3)
    assert torch.equal(Q1, s.get_state().cpu())
    s.close()


def _classic4(case):
    case.scheme.rk_scheme = "classic4"
    case.scheme.rk_stages = 4
    return case


CLASSIC4_CASES = {
    "box3d_20x18x16": lambda: synth.jittered_periodic_box(dims=(20, 18, 16), seed=3),
    "ramp_64x40": lambda: synth.compression_ramp(64, 40),
    "patchwork_3x2": lambda: synth.patchwork(seed=3, nbx=3, nby=2, side_lo=10, side_hi=30, h=1.0 / 48),
    "ramp_local_dt": lambda: synth.compression_ramp(48, 32, limiter="vanalbada"),
    "ns_box3d_20x18x16": lambda: _ns(synth.jittered_periodic_box(dims=(20, 18, 16), seed=5), 0.01),
}


def _ns(case, mu):
    case.scheme.viscosity = mu
    case.name += "_ns"
    return case


@pytest.mark.parametrize("name", sorted(CLASSIC4_CASES))
def test_classic4_matches_oracle(name):
    """CFD_RK_CLASSIC4 (classical fourth-order Runge-Kutta): 12 steps, state
    and per-step time step against the oracle's textbook implementation."""
    case = _classic4(CLASSIC4_CASES[name]())
    if name == "ramp_local_dt":
        case.scheme.local_dt = True
    Qref, dref = oracle_run(case, 12)
    s = _solver(case)
    dt = torch.empty(1, dtype=torch.float64, device="cuda:0")
    dts = []
    for _ in range(12):
        s.rk_step(1, dt)
        dts.append(dt.item())
    ok, rep = compare_state(s.get_state(), Qref, q_ref(case))
    _say("  classic4", name, rep)
    assert ok, rep
    assert max(abs(a - b) / b for a, b in zip(dts, dref)) <= 1e-12


def test_classic4_modes_bitwise_and_no_step_adjoint():
    """The classical scheme in every launch mode, both exchanges and with
    NaN-filled ghosts gives the same bits; the step adjoint and stage
    recording report CFD_ERR_UNSUPPORTED."""
    from paper_2012_02925_amd import capi
    case = _classic4(_rotated_two_block_box())
    outs = []
    for mode, graph, ghosts, flags in [("batched", True, "direct", 0), ("per_block", False, "direct", 0),
                                       ("persistent", True, "direct", 0), ("batched", False, "packed", 0),
                                       ("batched", False, "direct", capi.NAN_GHOSTS | capi.CHECK_FINITE)]:
        s = _solver(case, debug_flags=flags)
        s.set_exec(mode, graph)
        s.set_ghost_exchange(ghosts)
        s.rk_step(6)
        outs.append(((mode, graph, ghosts, flags), s.get_state().cpu()))
        s.close()
    for key, o in outs[1:]:
        assert torch.equal(outs[0][1], o), key
    ramp = _classic4(synth.compression_ramp(24, 16, dt_fixed=1e-3))
    s = _solver(ramp, adjoint=True)
    with pytest.raises(capi.CfdError) as e:
        s.rk_step_vjp(torch.zeros((ramp.nvar, ramp.ncells), dtype=torch.float64, device="cuda:0"))
    assert e.value.status == -7
    s.close()
