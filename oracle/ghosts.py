"""Ghost-cell fill: connected boundaries and physical boundary conditions.

Sec. 2: ghost cells enforce the boundary conditions and, for connected
boundaries, hold the neighbouring block's data so that every block can be
solved on its own.  Sec. 4 / Sec. 7.2 V1 and V5: connected-boundary data are
exchanged at every Runge-Kutta sub-iteration; a block may connect to itself
(the periodic case here).  Two ghost layers serve the four-cell MUSCL stencil
of eq. (flux).

Readings (the paper names the boundary types but prints no formulas):
  * connection: receiver ghost layer g (g = 1, 2 counted outward from the
    face) takes the donor's interior layer g (counted inward from its face)
    at the mapped tangential position;
  * slip wall: ghost layer g mirrors interior layer g: rho and p copied,
    velocity reflected about the wall face, u - 2 (u . n) n;
  * supersonic inflow: both ghost layers hold the inflow primitive state;
  * extrapolated outflow: both ghost layers copy the adjacent interior cell;
  * farfield, subsonic inflow, subsonic outflow: both ghost layers hold the
    characteristic boundary state of oracle/bc.py;
  * adiabatic no-slip wall: ghost layer g copies interior layer g with the
    velocity negated (rho and p copied, so T too).
Corner ghosts are not filled; the dimension-by-dimension stencil never reads them.

Arrays: interior primitive state ``q`` (nvar, [nk,] nj, ni); padded state
(nvar, [nk+4,] nj+4, ni+4).  Logical axis a (0 = i, 1 = j, 2 = k) is tensor
axis ``q.ndim - 1 - a``.
"""
import torch

from . import bc


def tensor_axis(ndim, logical_axis):
    return ndim - 1 - logical_axis


def tangential_axes(dim, face):
    return [a for a in range(dim) if a != face // 2]


def _to_logical_order(slab, dim):
    # slab has the normal axis removed; its non-variable axes are in
    # descending logical order; return (nvar, t1, t2) with t1 < t2 logical.
    if dim == 3:
        return slab.permute(0, 2, 1)
    return slab


def _from_logical_order(slab, dim):
    if dim == 3:
        return slab.permute(0, 2, 1)
    return slab


def interior_layer(q, dim, face, layer, lo, hi):
    """Interior cells ``layer`` cells in from ``face`` (0 = adjacent), over the
    tangential range [lo, hi); returned as (nvar, t1[, t2])."""
    axis = face // 2
    n = q.shape[tensor_axis(q.ndim, axis)]
    idx = layer if face % 2 == 0 else n - 1 - layer
    sl = [slice(None)] * q.ndim
    sl[tensor_axis(q.ndim, axis)] = idx
    for t, a in enumerate(tangential_axes(dim, face)):
        sl[tensor_axis(q.ndim, a)] = slice(lo[t], hi[t])
    return _to_logical_order(q[tuple(sl)], dim)


def face_area_slab(S_axis, dim, face, lo, hi):
    """Area vectors (dim, t1[, t2]) of the boundary faces of ``face`` over the range."""
    axis = face // 2
    ta = tensor_axis(S_axis.ndim, axis)
    idx = 0 if face % 2 == 0 else S_axis.shape[ta] - 1
    sl = [slice(None)] * S_axis.ndim
    sl[ta] = idx
    for t, a in enumerate(tangential_axes(dim, face)):
        sl[tensor_axis(S_axis.ndim, a)] = slice(lo[t], hi[t])
    return _to_logical_order(S_axis[tuple(sl)], dim)


def set_ghost_layer(qpad, dim, face, g, lo, hi, values):
    """Write ``values`` (nvar, t1[, t2]) into ghost layer g (1 or 2) of ``face``."""
    axis = face // 2
    ta = tensor_axis(qpad.ndim, axis)
    m = qpad.shape[ta]  # n + 4
    idx = 2 - g if face % 2 == 0 else m - 3 + g
    sl = [slice(None)] * qpad.ndim
    sl[ta] = idx
    for t, a in enumerate(tangential_axes(dim, face)):
        sl[tensor_axis(qpad.ndim, a)] = slice(lo[t] + 2, hi[t] + 2)
    qpad[tuple(sl)] = _from_logical_order(values, dim)


def map_to_donor(values_donor, dim, recv_len, orient):
    """Re-index a donor slab (nvar, T1D[, T2D]) onto the receiver's
    tangential positions: receiver offset (r1, r2) reads donor offset
    (d1, d2) with (s1, s2) = (r2, r1) if orient & 4 else (r1, r2) and
    d_m = T_mD - 1 - s_m where bit m-1 of orient is set, else s_m."""
    if dim == 2:
        r1 = torch.arange(recv_len[0])
        d1 = values_donor.shape[1] - 1 - r1 if orient & 1 else r1
        return values_donor[:, d1]
    L1, L2 = recv_len
    r1, r2 = torch.meshgrid(torch.arange(L1), torch.arange(L2), indexing="ij")
    s1, s2 = (r2, r1) if orient & 4 else (r1, r2)
    d1 = values_donor.shape[1] - 1 - s1 if orient & 1 else s1
    d2 = values_donor.shape[2] - 1 - s2 if orient & 2 else s2
    return values_donor[:, d1, d2]


def mirror(q_int_layer, S_face):
    """Slip-wall image of a primitive layer about faces with area vectors S."""
    n = S_face / torch.sqrt((S_face * S_face).sum(0))
    vel = q_int_layer[1:-1]
    vn = (vel * n).sum(0)
    vel_g = vel - 2.0 * vn * n
    return torch.cat([q_int_layer[:1], vel_g, q_int_layer[-1:]])


def fill_ghosts(problem, q_list, S_list):
    """Padded primitive arrays with every connected and physical ghost layer
    filled from the interior states ``q_list``."""
    dim = problem.dim
    pads = []
    for q in q_list:
        shape = [q.shape[0]] + [s + 4 for s in q.shape[1:]]
        qp = torch.zeros(shape, dtype=q.dtype)
        inner = [slice(None)] + [slice(2, -2)] * dim
        qp[tuple(inner)] = q
        pads.append(qp)
    # connections first (each is symmetric: both sides receive)
    for c in problem.conns:
        recv_len_a = [h - l for l, h in zip(c.lo_a, c.hi_a)]
        recv_len_b = [h - l for l, h in zip(c.lo_b, c.hi_b)]
        for g in (1, 2):
            donor_b = interior_layer(q_list[c.block_b], dim, c.face_b, g - 1, c.lo_b, c.hi_b)
            set_ghost_layer(pads[c.block_a], dim, c.face_a, g, c.lo_a, c.hi_a,
                            map_to_donor(donor_b, dim, recv_len_a, c.orient))
            # reverse direction: invert the offset map explicitly
            donor_a = interior_layer(q_list[c.block_a], dim, c.face_a, g - 1, c.lo_a, c.hi_a)
            set_ghost_layer(pads[c.block_b], dim, c.face_b, g, c.lo_b, c.hi_b,
                            _inverse_map(donor_a, dim, recv_len_b, recv_len_a, c.orient))
    # then physical boundaries
    for p in problem.bcs:
        q = q_list[p.block]
        for g in (1, 2):
            if p.kind == "slip_wall":
                Sf = face_area_slab(S_list[p.block][p.face // 2], dim, p.face, p.lo, p.hi)
                vals = mirror(interior_layer(q, dim, p.face, g - 1, p.lo, p.hi), Sf)
            elif p.kind == "noslip_wall":
                lay = interior_layer(q, dim, p.face, g - 1, p.lo, p.hi)
                vals = torch.cat([lay[:1], -lay[1:-1], lay[-1:]])
            elif p.kind == "extrap_outflow":
                vals = interior_layer(q, dim, p.face, 0, p.lo, p.hi)
            elif p.kind == "sup_inflow":
                theta = problem.bc_params[p.index]
                ref = interior_layer(q, dim, p.face, 0, p.lo, p.hi)
                vals = theta.reshape([-1] + [1] * (ref.ndim - 1)).expand_as(ref)
            elif p.kind in ("farfield", "sub_inflow", "sub_outflow"):
                vals = boundary_state(problem, p, q, S_list[p.block])
            else:
                raise ValueError(p.kind)
            set_ghost_layer(pads[p.block], dim, p.face, g, p.lo, p.hi, vals)
    return pads


def outward_normal(S_list_block, dim, face, lo, hi):
    """Unit outward normal (dim, t1[, t2]) of a block face over the range (the
    stored area vectors point towards increasing index)."""
    Sf = face_area_slab(S_list_block[face // 2], dim, face, lo, hi)
    n = Sf / torch.sqrt((Sf * Sf).sum(0))
    return -n if face % 2 == 0 else n


def boundary_state(problem, p, q, S_block):
    """Characteristic boundary state of a farfield / subsonic patch."""
    dim, g = problem.dim, problem.gamma
    qi = interior_layer(q, dim, p.face, 0, p.lo, p.hi)
    prm = torch.as_tensor(p.params, dtype=qi.dtype)
    if p.kind == "sub_inflow":
        return bc.subsonic_inflow_state(qi, prm, g)
    n = outward_normal(S_block, dim, p.face, p.lo, p.hi)
    if p.kind == "farfield":
        return bc.farfield_state(qi, n, prm, g)
    return bc.subsonic_outflow_state(qi, n, prm[0], g)


def _inverse_map(values_a, dim, len_b, len_a, orient):
    """Slab for side b's ghosts from side a's interior slab, where ``orient``
    maps a-offsets to b-offsets (see map_to_donor)."""
    if dim == 2:
        r1 = torch.arange(len_a[0])
        d1 = len_b[0] - 1 - r1 if orient & 1 else r1
        # b position d1 receives a position r1
        return values_a[:, torch.argsort(d1)]
    L1, L2 = len_a
    r1, r2 = torch.meshgrid(torch.arange(L1), torch.arange(L2), indexing="ij")
    s1, s2 = (r2, r1) if orient & 4 else (r1, r2)
    d1 = len_b[0] - 1 - s1 if orient & 1 else s1
    d2 = len_b[1] - 1 - s2 if orient & 2 else s2
    flat_b = (d1 * len_b[1] + d2).reshape(-1)
    src = values_a.reshape(values_a.shape[0], -1)
    order = torch.argsort(flat_b)
    return src[:, order].reshape(values_a.shape[0], len_b[0], len_b[1])
