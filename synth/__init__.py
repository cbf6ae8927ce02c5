"""Seeded synthetic inputs for the structured-grid Euler workloads.

This module only *describes* problems: node coordinates, block topology
(boundary patches and block-to-block connections), initial primitive fields
and the scheme settings a workload names.  It holds none of the solver's
arithmetic (no equation of state, no fluxes, no metrics) so that both the CPU
oracle and the GPU library can take their inputs from it without sharing any
part of the method.

Conventions shared by every consumer:

* Free stream is non-dimensionalised with rho_inf = 1, p_inf = 1/gamma (so the
  free-stream speed of sound is 1) and |V_inf| = Mach number.
* Node arrays are structure-of-arrays, ``nodes[c]`` is coordinate ``c`` and the
  remaining axes are ``(nk+1, nj+1, ni+1)`` in 3D or ``(nj+1, ni+1)`` in 2D
  (i fastest in memory).
* Cell arrays are ``(nvar, nk, nj, ni)`` / ``(nvar, nj, ni)``; primitive
  variables are ``(rho, u, v[, w], p)``.
* Faces of a block are numbered 0..5 = imin, imax, jmin, jmax, kmin, kmax.
  A patch range ``lo``/``hi`` is a half-open cell-index range along the face's
  tangential axes taken in increasing axis order (i before j before k).
* ``orient`` of a connection maps the receiving side's tangential offsets to
  the donor side's: bit 2 swaps the two tangential axes (3D only), bit 0
  reverses the donor's first tangential axis, bit 1 its second.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

GAMMA = 1.4

IMIN, IMAX, JMIN, JMAX, KMIN, KMAX = range(6)

SLIP_WALL = "slip_wall"
SUP_INFLOW = "sup_inflow"
EXTRAP_OUTFLOW = "extrap_outflow"
FARFIELD = "farfield"  # params: free-stream primitive state
SUB_INFLOW = "sub_inflow"  # params: (p0, rho0, direction)
SUB_OUTFLOW = "sub_outflow"  # params: (p_back,)
NOSLIP_WALL = "noslip_wall"  # adiabatic no-slip wall

LIMITER_NONE = "none"
LIMITER_VANLEER = "vanleer"
LIMITER_VANALBADA = "vanalbada"


@dataclasses.dataclass
class Block:
    ni: int
    nj: int
    nk: int  # 1 in 2D
    nodes: np.ndarray  # (dim, [nk+1,] nj+1, ni+1) float64


@dataclasses.dataclass
class BoundaryPatch:
    block: int
    face: int
    lo: Sequence[int]
    hi: Sequence[int]
    kind: str
    params: Optional[np.ndarray] = None  # per kind: see the kind constants above


@dataclasses.dataclass
class Connection:
    """Face range of block ``a`` abutting face range of block ``b``.

    Each side's ghost layers are filled from the other side's first interior
    layers; the connection is symmetric.
    """

    block_a: int
    face_a: int
    lo_a: Sequence[int]
    hi_a: Sequence[int]
    block_b: int
    face_b: int
    lo_b: Sequence[int]
    hi_b: Sequence[int]
    orient: int = 0


@dataclasses.dataclass
class Scheme:
    gamma: float = GAMMA
    limiter: str = LIMITER_VANLEER
    muscl_eps: float = 1.0
    muscl_kappa: float = -1.0
    # van Albada regularisation epsilon per primitive variable (rho, u, v[, w], p)
    lim_eps: Optional[Sequence[float]] = None
    efix: float = 0.1  # Harten smoothing width as a fraction of the Roe-averaged sound speed
    flux: str = "roe"  # "roe" | "vanleer_fvs" | "steger_warming"
    rk_stages: int = 4
    rk_scheme: str = "mstage"  # "mstage" (Sec. 2) or "classic4" (classical fourth-order Runge-Kutta)
    cfl: float = 0.5
    dt_fixed: Optional[float] = None  # None = global CFL time step recomputed every step
    local_dt: bool = False  # local time stepping: every cell with its own CFL step (steady runs)
    viscosity: float = 0.0  # laminar Navier-Stokes when > 0: mu = M_inf / Re in free-stream units
    prandtl: float = 0.72


@dataclasses.dataclass
class Case:
    name: str
    dim: int
    blocks: List[Block]
    bcs: List[BoundaryPatch]
    conns: List[Connection]
    prims: List[np.ndarray]  # initial primitive state per block
    scheme: Scheme
    steps: int
    meta: Dict = dataclasses.field(default_factory=dict)

    @property
    def nvar(self) -> int:
        return self.dim + 2

    @property
    def ncells(self) -> int:
        return sum(b.ni * b.nj * b.nk for b in self.blocks)


# ---------------------------------------------------------------------------
# topology helpers


def face_tangential_extent(dim: int, face: int, ni: int, nj: int, nk: int):
    """Cell counts along the tangential axes of ``face`` (increasing axis order)."""
    n = (ni, nj, nk)[:dim]
    axis = face // 2
    return [n[a] for a in range(dim) if a != axis]


def periodic_self_connections(dim: int, ni: int, nj: int, nk: int = 1, block: int = 0):
    """Connections that make a single block periodic in every index direction."""
    conns = []
    for axis in range(dim):
        ext = face_tangential_extent(dim, 2 * axis, ni, nj, nk)
        lo = [0] * (dim - 1)
        conns.append(Connection(block, 2 * axis, lo, ext, block, 2 * axis + 1, lo, ext, 0))
    return conns


def full_face_patch(case_dim: int, blk: Block, block: int, face: int, kind: str, params=None):
    ext = face_tangential_extent(case_dim, face, blk.ni, blk.nj, blk.nk)
    return BoundaryPatch(block, face, [0] * (case_dim - 1), ext, kind,
                         None if params is None else np.asarray(params, dtype=np.float64))


# ---------------------------------------------------------------------------
# grids


def cartesian_nodes_2d(ni: int, nj: int, x0=0.0, y0=0.0, hx=None, hy=None, lx=1.0, ly=1.0):
    hx = lx / ni if hx is None else hx
    hy = ly / nj if hy is None else hy
    x = x0 + hx * np.arange(ni + 1, dtype=np.float64)
    y = y0 + hy * np.arange(nj + 1, dtype=np.float64)
    X, Y = np.meshgrid(x, y, indexing="xy")  # (nj+1, ni+1)
    return np.stack([X, Y]).astype(np.float64)


def ramp_nodes_2d(ni: int, nj: int, length=1.5, corner=0.5, angle_deg=10.0, stretch=1.0):
    """Compression-ramp grid: x uniform on [0, length]; the lower wall turns by
    ``angle_deg`` at ``x = corner``; j-lines are algebraically stretched toward
    the wall with s(eta) = eta / (1 + stretch (1 - eta))."""
    x = length * np.arange(ni + 1, dtype=np.float64) / ni
    eta = np.arange(nj + 1, dtype=np.float64) / nj
    s = eta / (1.0 + stretch * (1.0 - eta))
    yw = np.where(x <= corner, 0.0, (x - corner) * math.tan(math.radians(angle_deg)))
    X = np.broadcast_to(x[None, :], (nj + 1, ni + 1)).copy()
    Y = yw[None, :] + (1.0 - yw[None, :]) * s[:, None]
    return np.stack([X, Y]).astype(np.float64)


def _random_wavevectors(rng, count, dim, kmax=3):
    out = []
    while len(out) < count:
        k = rng.integers(-kmax, kmax + 1, size=dim)
        if np.any(k != 0):
            out.append(k)
    return np.array(out, dtype=np.float64)


def jittered_periodic_nodes_3d(ni: int, nj: int, nk: int, seed: int, amp=0.05, nmodes=4):
    """Unit-cube nodes displaced by a smooth periodic field of amplitude
    ``amp`` times the local spacing in each component (never more)."""
    rng = np.random.default_rng(seed)
    h = (1.0 / ni, 1.0 / nj, 1.0 / nk)
    xs = [np.arange(n + 1, dtype=np.float64) / n for n in (ni, nj, nk)]
    # broadcastable coordinate axes in (k, j, i) order
    X = xs[0][None, None, :]
    Y = xs[1][None, :, None]
    Z = xs[2][:, None, None]
    out = np.empty((3, nk + 1, nj + 1, ni + 1), dtype=np.float64)
    base = (X, Y, Z)
    for c in range(3):
        ks = _random_wavevectors(rng, nmodes, 3)
        ph = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
        J = np.zeros((nk + 1, nj + 1, ni + 1), dtype=np.float64)
        for m in range(nmodes):
            J += np.sin(2.0 * np.pi * (ks[m, 0] * X + ks[m, 1] * Y + ks[m, 2] * Z) + ph[m])
        J /= nmodes
        out[c] = np.broadcast_to(base[c], J.shape) + amp * h[c] * J
    return out


def jittered_periodic_nodes_2d(ni: int, nj: int, seed: int, amp=0.05, nmodes=4):
    rng = np.random.default_rng(seed)
    h = (1.0 / ni, 1.0 / nj)
    X = (np.arange(ni + 1, dtype=np.float64) / ni)[None, :]
    Y = (np.arange(nj + 1, dtype=np.float64) / nj)[:, None]
    out = np.empty((2, nj + 1, ni + 1), dtype=np.float64)
    for c, B in enumerate((X, Y)):
        ks = _random_wavevectors(rng, nmodes, 2)
        ph = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
        J = np.zeros((nj + 1, ni + 1))
        for m in range(nmodes):
            J += np.sin(2.0 * np.pi * (ks[m, 0] * X + ks[m, 1] * Y) + ph[m])
        out[c] = np.broadcast_to(B, J.shape) + amp * h[c] * J / nmodes
    return out


def cell_centres_index_space(ni, nj, nk=None, lx=1.0, ly=1.0, lz=1.0):
    """Undisplaced cell centres (used to sample initial fields)."""
    x = (np.arange(ni) + 0.5) * lx / ni
    y = (np.arange(nj) + 0.5) * ly / nj
    if nk is None:
        return np.meshgrid(x, y, indexing="xy")
    z = (np.arange(nk) + 0.5) * lz / nk
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


# ---------------------------------------------------------------------------
# workloads


def gaussian_bump_periodic(ni=64, nj=64, seed=0, mach=0.5, amp=0.01, sigma=0.1,
                           limiter=LIMITER_VANLEER, steps=100) -> Case:
    """2D periodic unit square, free stream along +x plus a Gaussian density
    bump (summed over the nearest periodic images so it is smooth across the
    seam); pressure and velocity uniform."""
    rng = np.random.default_rng(seed)
    xc = rng.uniform(0.0, 1.0, size=2)
    X, Y = cell_centres_index_space(ni, nj)
    rho = np.ones_like(X)
    for m in (-1, 0, 1):
        for n in (-1, 0, 1):
            d2 = (X - xc[0] - m) ** 2 + (Y - xc[1] - n) ** 2
            rho += amp * np.exp(-d2 / (2.0 * sigma ** 2))
    prim = np.stack([rho, np.full_like(X, mach), np.zeros_like(X), np.full_like(X, 1.0 / GAMMA)])
    blk = Block(ni, nj, 1, cartesian_nodes_2d(ni, nj))
    return Case("gaussian_bump_periodic_%dx%d" % (ni, nj), 2, [blk], [],
                periodic_self_connections(2, ni, nj), [prim],
                Scheme(limiter=limiter), steps, meta={"bump_centre": xc, "mach": mach})


def compression_ramp(ni=1024, nj=1024, mach=2.5, limiter=LIMITER_VANLEER, steps=500,
                     lim_eps=None, dt_fixed=None, inflow=None) -> Case:
    """2D supersonic flow over a 10-degree compression ramp: supersonic inflow
    at imin, extrapolated outflow at imax and jmax, slip wall at jmin; the
    flow starts as the uniform inflow state."""
    nodes = ramp_nodes_2d(ni, nj)
    blk = Block(ni, nj, 1, nodes)
    theta = np.array([1.0, mach, 0.0, 1.0 / GAMMA]) if inflow is None else np.asarray(inflow, float)
    bcs = [full_face_patch(2, blk, 0, IMIN, SUP_INFLOW, theta),
           full_face_patch(2, blk, 0, IMAX, EXTRAP_OUTFLOW),
           full_face_patch(2, blk, 0, JMIN, SLIP_WALL),
           full_face_patch(2, blk, 0, JMAX, EXTRAP_OUTFLOW)]
    prim = np.broadcast_to(theta[:, None, None], (4, nj, ni)).copy()
    sch = Scheme(limiter=limiter, lim_eps=lim_eps, dt_fixed=dt_fixed)
    return Case("compression_ramp_%dx%d" % (ni, nj), 2, [blk], bcs, [], [prim], sch, steps,
                meta={"inflow": theta})


def jittered_periodic_box(n=256, seed=0, mach=0.8, amp=0.02, nmodes=4,
                          limiter=LIMITER_VANALBADA, steps=50, dims=None) -> Case:
    """3D periodic unit cube on a smoothly jittered grid; free stream along +x
    plus random-phase sinusoidal velocity perturbations."""
    ni, nj, nk = (n, n, n) if dims is None else dims
    nodes = jittered_periodic_nodes_3d(ni, nj, nk, seed)
    rng = np.random.default_rng(seed + 7919)
    X, Y, Z = cell_centres_index_space(ni, nj, nk)
    vel = [np.full_like(X, mach), np.zeros_like(X), np.zeros_like(X)]
    for c in range(3):
        ks = _random_wavevectors(rng, nmodes, 3)
        ph = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
        pert = np.zeros_like(X)
        for m in range(nmodes):
            pert += np.sin(2.0 * np.pi * (ks[m, 0] * X + ks[m, 1] * Y + ks[m, 2] * Z) + ph[m])
        vel[c] = vel[c] + amp * mach * pert / nmodes
    prim = np.stack([np.ones_like(X), vel[0], vel[1], vel[2], np.full_like(X, 1.0 / GAMMA)])
    blk = Block(ni, nj, nk, nodes)
    sch = Scheme(limiter=limiter, lim_eps=[0.0] * 5)
    return Case("jittered_periodic_box_%dx%dx%d" % (ni, nj, nk), 3, [blk], [],
                periodic_self_connections(3, ni, nj, nk), [prim], sch, steps)


def jittered_periodic_square(ni=64, nj=64, seed=0, mach=0.8, amp=0.02, nmodes=4,
                             limiter=LIMITER_VANALBADA, steps=50) -> Case:
    """2D analogue of :func:`jittered_periodic_box` (used for conservation and
    freestream-preservation checks on curved periodic grids)."""
    nodes = jittered_periodic_nodes_2d(ni, nj, seed)
    rng = np.random.default_rng(seed + 7919)
    X, Y = cell_centres_index_space(ni, nj)
    vel = [np.full_like(X, mach), np.zeros_like(X)]
    for c in range(2):
        ks = _random_wavevectors(rng, nmodes, 2)
        ph = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
        pert = np.zeros_like(X)
        for m in range(nmodes):
            pert += np.sin(2.0 * np.pi * (ks[m, 0] * X + ks[m, 1] * Y) + ph[m])
        vel[c] = vel[c] + amp * mach * pert / nmodes
    prim = np.stack([np.ones_like(X), vel[0], vel[1], np.full_like(X, 1.0 / GAMMA)])
    blk = Block(ni, nj, 1, nodes)
    sch = Scheme(limiter=limiter, lim_eps=[0.0] * 4)
    return Case("jittered_periodic_square_%dx%d" % (ni, nj), 2, [blk], [],
                periodic_self_connections(2, ni, nj), [prim], sch, steps)


def patchwork(seed=0, nbx=8, nby=8, side_lo=64, side_hi=512, h=1.0 / 512, mach=2.0,
              amp=0.01, nmodes=4, limiter=LIMITER_VANLEER, steps=200) -> Case:
    """2D periodic patchwork of ``nbx * nby`` Cartesian blocks whose column
    widths and row heights are drawn uniformly from [side_lo, side_hi]; every
    block face is connected 1:1 to its neighbour (wrapping at the outer
    boundary), so all faces are connections."""
    rng = np.random.default_rng(seed)
    widths = rng.integers(side_lo, side_hi + 1, size=nbx)
    heights = rng.integers(side_lo, side_hi + 1, size=nby)
    x0 = np.concatenate([[0], np.cumsum(widths)]) * h
    y0 = np.concatenate([[0], np.cumsum(heights)]) * h
    Lx, Ly = x0[-1], y0[-1]
    ks = _random_wavevectors(rng, nmodes, 2)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=nmodes)
    blocks, prims = [], []
    bid = lambda a, b: b * nbx + a
    for b in range(nby):
        for a in range(nbx):
            ni, nj = int(widths[a]), int(heights[b])
            blocks.append(Block(ni, nj, 1, cartesian_nodes_2d(ni, nj, x0[a], y0[b], h, h)))
            X = x0[a] + (np.arange(ni) + 0.5)[None, :] * h + 0.0 * np.arange(nj)[:, None]
            Y = y0[b] + (np.arange(nj) + 0.5)[:, None] * h + 0.0 * np.arange(ni)[None, :]
            rho = np.ones((nj, ni))
            for m in range(nmodes):
                rho += amp * np.sin(2 * np.pi * (ks[m, 0] * X / Lx + ks[m, 1] * Y / Ly) + ph[m]) / nmodes
            prims.append(np.stack([rho, np.full_like(rho, mach), np.zeros_like(rho),
                                   np.full_like(rho, 1.0 / GAMMA)]))
    conns = []
    for b in range(nby):
        for a in range(nbx):
            A = bid(a, b)
            E = bid((a + 1) % nbx, b)
            N = bid(a, (b + 1) % nby)
            hA, wA = int(heights[b]), int(widths[a])
            conns.append(Connection(A, IMAX, [0], [hA], E, IMIN, [0], [hA], 0))
            conns.append(Connection(A, JMAX, [0], [wA], N, JMIN, [0], [wA], 0))
    return Case("patchwork_%dx%d_seed%d" % (nbx, nby, seed), 2, blocks, [], conns, prims,
                Scheme(limiter=limiter), steps, meta={"widths": widths, "heights": heights})


def stagnation_state(mach, gamma=GAMMA, rho=1.0, p=1.0 / GAMMA):
    """Stagnation pressure and density of a flow at Mach ``mach`` with static
    density ``rho`` and pressure ``p`` (isentropic relations)."""
    f = 1.0 + 0.5 * (gamma - 1.0) * mach * mach
    return p * f ** (gamma / (gamma - 1.0)), rho * f ** (1.0 / (gamma - 1.0))


def _smooth_field(rng, X, Y, nmodes=3, Z=None):
    """Sum of random low-wavenumber cosines scaled to max |f| <= 1."""
    f = np.zeros_like(X)
    for _ in range(nmodes):
        k = rng.integers(1, 4, size=3)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        arg = np.pi * (k[0] * X + k[1] * Y + (0.0 if Z is None else k[2] * Z)) + ph
        f += np.cos(arg)
    return f / nmodes


def bump_channel_nodes_2d(ni, nj, length=3.0, height=1.0, bump=0.1, jitter=0.0, seed=0):
    """Channel [0, length] x [0, height] whose lower wall carries a sin^2 bump
    of height ``bump`` between x = length/3 and 2 length/3; nodes spread
    uniformly between the walls, interior nodes optionally moved in index
    space by a smooth seeded field of amplitude ``jitter`` (a fraction of the
    domain; it vanishes on the boundary)."""
    xi = np.linspace(0.0, 1.0, ni + 1)
    eta = np.linspace(0.0, 1.0, nj + 1)
    XI, ETA = np.meshgrid(xi, eta, indexing="xy")
    if jitter:
        rng = np.random.default_rng(seed)
        fx = _smooth_field(rng, XI, ETA) * np.sin(np.pi * XI) * np.sin(np.pi * ETA)
        fy = _smooth_field(rng, XI, ETA) * np.sin(np.pi * XI) * np.sin(np.pi * ETA)
        XI = XI + jitter * fx
        ETA = ETA + jitter * fy
    X = length * XI
    a, b = length / 3.0, 2.0 * length / 3.0
    yw = np.where((X > a) & (X < b), bump * np.sin(np.pi * (X - a) / (b - a)) ** 2, 0.0)
    Y = yw + (height - yw) * ETA
    return np.stack([X, Y]).astype(np.float64)


def subsonic_channel(ni=96, nj=32, mach=0.5, seed=0, amp=0.02, pressure_amp=0.0,
                     limiter=LIMITER_VANLEER, steps=200) -> Case:
    """2D channel with a bump on the lower wall: subsonic inflow at imin
    (stagnation state of the Mach ``mach`` free stream, direction +x),
    subsonic outflow at imax (back pressure 1/gamma), slip walls at jmin and
    jmax.  Initial state: the free stream plus smooth seeded perturbations of
    velocity (``amp`` of the free-stream speed) and pressure
    (``pressure_amp`` of the static pressure)."""
    nodes = bump_channel_nodes_2d(ni, nj, jitter=0.02, seed=seed)
    blk = Block(ni, nj, 1, nodes)
    p0, r0 = stagnation_state(mach)
    rng = np.random.default_rng(seed + 101)
    X, Y = cell_centres_index_space(ni, nj)
    u = mach * (1.0 + amp * _smooth_field(rng, X, Y))
    v = mach * amp * _smooth_field(rng, X, Y)
    p = (1.0 + pressure_amp * _smooth_field(rng, X, Y)) / GAMMA
    prim = np.stack([np.ones_like(X) + 0.5 * amp * _smooth_field(rng, X, Y), u, v, p])
    bcs = [full_face_patch(2, blk, 0, IMIN, SUB_INFLOW, [p0, r0, 1.0, 0.0]),
           full_face_patch(2, blk, 0, IMAX, SUB_OUTFLOW, [1.0 / GAMMA]),
           full_face_patch(2, blk, 0, JMIN, SLIP_WALL),
           full_face_patch(2, blk, 0, JMAX, SLIP_WALL)]
    return Case("subsonic_channel_%dx%d" % (ni, nj), 2, [blk], bcs, [], [prim],
                Scheme(limiter=limiter), steps, meta={"p0": p0, "rho0": r0, "mach": mach})


def farfield_bump(ni=96, nj=48, mach=0.6, alpha_deg=3.0, seed=0, amp=0.05,
                  limiter=LIMITER_VANLEER, steps=200) -> Case:
    """2D flow over a bump in a box [0, 3] x [0, 1.5]: farfield at imin, imax
    and jmax (free stream at Mach ``mach``, angle ``alpha_deg``), slip wall at
    jmin.  Initial state: the free stream plus smooth seeded perturbations of
    relative amplitude ``amp``, so that the boundary sees inflow and outflow
    and both signs of the boundary normal velocity."""
    nodes = bump_channel_nodes_2d(ni, nj, height=1.5, bump=0.08, jitter=0.02, seed=seed)
    blk = Block(ni, nj, 1, nodes)
    a = np.deg2rad(alpha_deg)
    qinf = np.array([1.0, mach * np.cos(a), mach * np.sin(a), 1.0 / GAMMA])
    rng = np.random.default_rng(seed + 202)
    X, Y = cell_centres_index_space(ni, nj)
    prim = np.stack([qinf[0] * (1.0 + amp * _smooth_field(rng, X, Y)),
                     qinf[1] + mach * amp * _smooth_field(rng, X, Y),
                     qinf[2] + mach * amp * _smooth_field(rng, X, Y),
                     qinf[3] * (1.0 + amp * _smooth_field(rng, X, Y))])
    bcs = [full_face_patch(2, blk, 0, IMIN, FARFIELD, qinf),
           full_face_patch(2, blk, 0, IMAX, FARFIELD, qinf),
           full_face_patch(2, blk, 0, JMIN, SLIP_WALL),
           full_face_patch(2, blk, 0, JMAX, FARFIELD, qinf)]
    return Case("farfield_bump_%dx%d_M%g" % (ni, nj, mach), 2, [blk], bcs, [], [prim],
                Scheme(limiter=limiter), steps, meta={"qinf": qinf})


def characteristic_box_3d(dims=(40, 24, 20), seed=0, mach=0.5, amp=0.03,
                          limiter=LIMITER_VANALBADA, steps=50) -> Case:
    """3D box on a jittered grid exercising every characteristic boundary:
    subsonic inflow at imin (direction tilted off the i axis), subsonic
    outflow at imax, slip wall at jmin, farfield at jmax and kmin,
    extrapolation at kmax.  Initial state: the free stream plus smooth seeded
    perturbations."""
    ni, nj, nk = dims
    nodes = jittered_periodic_nodes_3d(ni, nj, nk, seed)
    blk = Block(ni, nj, nk, nodes)
    d = np.array([1.0, 0.1, 0.05])
    qinf = np.array([1.0, mach, 0.0, 0.0, 1.0 / GAMMA])
    p0, r0 = stagnation_state(mach)
    rng = np.random.default_rng(seed + 303)
    X, Y, Z = cell_centres_index_space(ni, nj, nk)
    prim = np.stack([1.0 + amp * _smooth_field(rng, X, Y, Z=Z),
                     mach * (1.0 + amp * _smooth_field(rng, X, Y, Z=Z)),
                     mach * amp * _smooth_field(rng, X, Y, Z=Z),
                     mach * amp * _smooth_field(rng, X, Y, Z=Z),
                     (1.0 + amp * _smooth_field(rng, X, Y, Z=Z)) / GAMMA])
    bcs = [full_face_patch(3, blk, 0, IMIN, SUB_INFLOW, [p0, r0, *(d / np.sqrt((d * d).sum()))]),
           full_face_patch(3, blk, 0, IMAX, SUB_OUTFLOW, [1.0 / GAMMA]),
           full_face_patch(3, blk, 0, JMIN, SLIP_WALL),
           full_face_patch(3, blk, 0, JMAX, FARFIELD, qinf),
           full_face_patch(3, blk, 0, KMIN, FARFIELD, qinf),
           full_face_patch(3, blk, 0, KMAX, EXTRAP_OUTFLOW)]
    sch = Scheme(limiter=limiter, lim_eps=[0.0] * 5)
    return Case("characteristic_box_%dx%dx%d" % (ni, nj, nk), 3, [blk], bcs, [], [prim], sch, steps,
                meta={"qinf": qinf, "p0": p0, "rho0": r0})


def split_block_case(case: Case, splits_i: Sequence[int], splits_j: Sequence[int]) -> Case:
    """Split the single 2D block of ``case`` at the given i and j cell indices
    into a grid of connected sub-blocks.  Physical patches and connections of
    the parent that span whole faces are re-linked to the sub-blocks."""
    assert case.dim == 2 and len(case.blocks) == 1
    parent = case.blocks[0]
    ib = [0] + list(splits_i) + [parent.ni]
    jb = [0] + list(splits_j) + [parent.nj]
    na, nb = len(ib) - 1, len(jb) - 1
    blocks, prims = [], []
    bid = lambda a, b: b * na + a
    for b in range(nb):
        for a in range(na):
            i0, i1, j0, j1 = ib[a], ib[a + 1], jb[b], jb[b + 1]
            blocks.append(Block(i1 - i0, j1 - j0, 1, parent.nodes[:, j0:j1 + 1, i0:i1 + 1].copy()))
            prims.append(case.prims[0][:, j0:j1, i0:i1].copy())
    conns = []
    for b in range(nb):
        for a in range(na):
            if a + 1 < na:
                h = jb[b + 1] - jb[b]
                conns.append(Connection(bid(a, b), IMAX, [0], [h], bid(a + 1, b), IMIN, [0], [h]))
            if b + 1 < nb:
                w = ib[a + 1] - ib[a]
                conns.append(Connection(bid(a, b), JMAX, [0], [w], bid(a, b + 1), JMIN, [0], [w]))

    def sub_of(face, t):  # which sub-block segment along the face's tangential axis
        bounds = jb if face in (IMIN, IMAX) else ib
        segs = []
        for s in range(len(bounds) - 1):
            segs.append((bounds[s], bounds[s + 1]))
        return segs

    # parent periodic self-connections become connections between edge blocks
    for c in case.conns:
        assert c.block_a == 0 and c.block_b == 0 and c.orient == 0
        for s, (t0, t1) in enumerate(sub_of(c.face_a, None)):
            if c.face_a == IMIN:
                A, B = bid(0, s), bid(na - 1, s)
            elif c.face_a == JMIN:
                A, B = bid(s, 0), bid(s, nb - 1)
            else:
                raise ValueError("split supports imin/jmin-anchored periodic connections")
            conns.append(Connection(A, c.face_a, [0], [t1 - t0], B, c.face_b, [0], [t1 - t0]))
    bcs = []
    for p in case.bcs:
        for s, (t0, t1) in enumerate(sub_of(p.face, None)):
            if p.face == IMIN:
                blk = bid(0, s)
            elif p.face == IMAX:
                blk = bid(na - 1, s)
            elif p.face == JMIN:
                blk = bid(s, 0)
            else:
                blk = bid(s, nb - 1)
            bcs.append(BoundaryPatch(blk, p.face, [0], [t1 - t0], p.kind, p.params))
    return Case(case.name + "_split", 2, blocks, bcs, conns, prims, case.scheme, case.steps,
                meta=dict(case.meta))


# ---------------------------------------------------------------------------
# directions for derivative checks


def inflow_directions(count: int, seed: int, nvar: int = 4):
    """Seeded unit-norm directions in the space of inflow primitive states."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((count, nvar))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def node_displacement_fields(block: Block, count: int, seed: int, nmodes=3):
    """Smooth node displacement fields (2D), proportional to the local node
    spacing, nonzero on the wall and in the interior alike, scaled so the
    largest displacement component of each field is 1."""
    rng = np.random.default_rng(seed)
    nodes = block.nodes
    nj1, ni1 = nodes.shape[1], nodes.shape[2]
    s = (np.arange(ni1) / (ni1 - 1))[None, :]
    t = (np.arange(nj1) / (nj1 - 1))[:, None]
    # local spacing from the node array itself (geometry input, not a metric)
    hx = np.gradient(nodes[0], axis=1)
    hy = np.gradient(nodes[1], axis=0)
    out = np.empty((count,) + nodes.shape)
    for n in range(count):
        for c, hc in enumerate((hx, hy)):
            f = np.zeros((nj1, ni1))
            for m in range(nmodes):
                a, b = rng.integers(1, 4, size=2)
                ph = rng.uniform(0, 2 * np.pi, size=2)
                f += np.sin(np.pi * a * s + ph[0]) * np.cos(np.pi * b * t + ph[1])
            out[n, c] = np.abs(hc) * f
        out[n] /= np.abs(out[n]).max()
    return out


WORKLOADS = {
    "gaussian_bump_periodic": gaussian_bump_periodic,
    "compression_ramp": compression_ramp,
    "jittered_periodic_box": jittered_periodic_box,
    "patchwork": patchwork,
}
