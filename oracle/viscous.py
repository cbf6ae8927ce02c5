"""Laminar viscous flux: Green's theorem face gradients and the viscous residual.

Sec. 2, eq. (governing): the residual carries the viscous normal flux
F_v,n = (0, tau . n, Theta . n) with the Stokes-hypothesis stresses and
Theta_i = u_j tau_ij + k dT/dx_i; the face gradients come from Green's theorem
on a stencil wider than the inviscid one.  The paper prints no formulas; the
readings here:

* Units: rho_inf = 1, c_inf = 1, p_inf = 1/gamma; temperature T = gamma p / rho
  (T_inf = 1, gas constant 1/gamma, c_p = 1/(gamma - 1)); constant viscosity
  mu (mu = M_inf / Re for a Reynolds number Re per unit length); conductivity
  k = mu c_p / Pr.
* Stresses: tau = mu (grad u + grad u^T) - 2/3 mu (div u) I.
* Face gradients: Green's theorem over the dual volume of the face, the
  polygon (2D) or double pyramid (3D) spanned by the two cell centres beside
  the face and the face's corner "pseudo-nodes".  A pseudo-node carries the
  mean position and the mean value of the cells around the grid node that are
  interior or face ghosts (edge and corner ghosts are never formed); with
  vertex values averaged along each edge (2D) or over each triangle (3D) the
  gradient is exact for fields linear in space.
* Face values of u and T for Theta: the mean of the two cells beside the face.
* Cell centres: mean of the cell's nodes.  First-layer ghost centres: at a
  connection the donor's centre moved by the offset between the two sides'
  face centres (so translation-periodic blocks work); at a physical boundary
  the interior centre mirrored in the plane of the boundary face.
* Viscous residual Rv = (1/Omega) sum over faces F_v . S_out; the total
  residual is R = R_inviscid - Rv.

TEST INFRASTRUCTURE ONLY (part of the oracle).
"""
import itertools

import torch

from .ghosts import (_inverse_map, face_area_slab, interior_layer, map_to_donor, set_ghost_layer,
                     tangential_axes, tensor_axis)


def cell_centers(X):
    """Mean of each cell's 2^dim nodes: (dim, [nk,] nj, ni)."""
    dim = X.shape[0]
    acc = 0.0
    for offs in itertools.product((0, 1), repeat=dim):
        sl = [slice(None)]
        for ta in range(dim):
            o = offs[ta]
            sl.append(slice(o, X.shape[1 + ta] - 1 + o))
        acc = acc + X[tuple(sl)]
    return acc / (2 ** dim)


def face_centers(X, dim, face, lo, hi):
    """Mean of the nodes of every boundary face of ``face`` over the cell
    range [lo, hi): (dim, t1[, t2]) in increasing logical axis order."""
    axis = face // 2
    nd = X.ndim
    n = X.shape[tensor_axis(nd, axis)] - 1
    sl_base = [slice(None)] * nd
    sl_base[tensor_axis(nd, axis)] = 0 if face % 2 == 0 else n
    tang = tangential_axes(dim, face)
    acc = 0.0
    for offs in itertools.product((0, 1), repeat=dim - 1):
        sl = list(sl_base)
        for t, a in enumerate(tang):
            sl[tensor_axis(nd, a)] = slice(lo[t] + offs[t], hi[t] + offs[t])
        acc = acc + X[tuple(sl)]
    acc = acc / (2 ** (dim - 1))
    return acc.permute(0, 2, 1) if dim == 3 else acc


def padded_centers(problem, X_list, S_list):
    """Cell centres in the padded layout with the first ghost layer of every
    block face filled (see the module readings); other ghosts are zero."""
    dim = problem.dim
    C = [cell_centers(X) for X in X_list]
    pads = []
    for c in C:
        shape = [dim] + [s + 4 for s in c.shape[1:]]
        p = torch.zeros(shape, dtype=c.dtype)
        p[tuple([slice(None)] + [slice(2, -2)] * dim)] = c
        pads.append(p)
    for cn in problem.conns:
        la = [h - l for l, h in zip(cn.lo_a, cn.hi_a)]
        lb = [h - l for l, h in zip(cn.lo_b, cn.hi_b)]
        fa = face_centers(X_list[cn.block_a], dim, cn.face_a, cn.lo_a, cn.hi_a)
        fb = face_centers(X_list[cn.block_b], dim, cn.face_b, cn.lo_b, cn.hi_b)
        rel_b = interior_layer(C[cn.block_b], dim, cn.face_b, 0, cn.lo_b, cn.hi_b) - fb
        set_ghost_layer(pads[cn.block_a], dim, cn.face_a, 1, cn.lo_a, cn.hi_a, fa + map_to_donor(rel_b, dim, la, cn.orient))
        rel_a = interior_layer(C[cn.block_a], dim, cn.face_a, 0, cn.lo_a, cn.hi_a) - fa
        set_ghost_layer(pads[cn.block_b], dim, cn.face_b, 1, cn.lo_b, cn.hi_b,
                        fb + _inverse_map(rel_a, dim, lb, la, cn.orient))
    for p in problem.bcs:
        X = X_list[p.block]
        fc = face_centers(X, dim, p.face, p.lo, p.hi)
        Sf = face_area_slab(S_list[p.block][p.face // 2], dim, p.face, p.lo, p.hi)
        n = Sf / torch.sqrt((Sf * Sf).sum(0))
        c0 = interior_layer(C[p.block], dim, p.face, 0, p.lo, p.hi)
        set_ghost_layer(pads[p.block], dim, p.face, 1, p.lo, p.hi, c0 - 2.0 * ((c0 - fc) * n).sum(0) * n)
    return pads


def pseudo_nodes(pad, dim):
    """Mean over the cells around every grid node that are interior or face
    ghosts (at most one index outside the block): (c, [nk+1,] nj+1, ni+1)."""
    nd = pad.ndim
    ncell = [pad.shape[tensor_axis(nd, a)] - 4 for a in range(dim)]
    total, count = 0.0, 0.0
    for offs in itertools.product((0, 1), repeat=dim):  # offs[a]: cell index node - 1 + offs[a]
        sl = [slice(None)] * nd
        outside = 0
        for a in range(dim):
            ta = tensor_axis(nd, a)
            sl[ta] = slice(1 + offs[a], 1 + offs[a] + ncell[a] + 1)
            idx = torch.arange(ncell[a] + 1)
            out_a = (idx == 0) if offs[a] == 0 else (idx == ncell[a])
            shape = [1] * (nd - 1)
            shape[ta - 1] = ncell[a] + 1
            outside = outside + out_a.reshape(shape).to(torch.int64)
        ok = (outside <= 1)
        vals = pad[tuple(sl)]
        total = total + torch.where(ok, vals, torch.zeros_like(vals))
        count = count + ok.to(pad.dtype)
    return total / count


def _cross(a, b):
    return torch.stack([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def face_gradients(padC, padV, nodeP, nodeV, dim, d):
    """Green's-theorem gradients on every face of direction d (faces 0..n_d,
    interior range along the other directions).  padC/padV: padded cell
    centres/values; nodeP/nodeV: pseudo-node positions/values.  Returns
    (c, dim, faces...) with [:, k] the derivative along x_k."""
    nd = padC.ndim
    ta = tensor_axis(nd, d)

    def cells(start):
        sl = [slice(None)] * nd
        for a in range(dim):
            if a == d:
                sl[tensor_axis(nd, a)] = slice(start, padC.shape[ta] - 4 + start + 1)
            else:
                sl[tensor_axis(nd, a)] = slice(2, -2)
        return tuple(sl)

    def node(offs):
        sl = [slice(None)] * nd
        for t, a in enumerate([x for x in range(dim) if x != d]):
            n_a = nodeP.shape[tensor_axis(nd, a)] - 1
            sl[tensor_axis(nd, a)] = slice(offs[t], n_a + offs[t])
        return tuple(sl)

    CL, CR = padC[cells(1)], padC[cells(2)]
    VL, VR = padV[cells(1)], padV[cells(2)]
    if dim == 2:
        verts = [(CL, VL), (nodeP[node((0,))], nodeV[node((0,))]), (CR, VR), (nodeP[node((1,))], nodeV[node((1,))])]
        A = 0.0
        G = 0.0
        for k in range(4):
            (pa, va), (pb, vb) = verts[k], verts[(k + 1) % 4]
            A = A + 0.5 * (pa[0] * pb[1] - pb[0] * pa[1])
            m = torch.stack([pb[1] - pa[1], -(pb[0] - pa[0])])  # edge normal times length
            G = G + 0.5 * (va + vb)[:, None] * m[None]
        return G / A
    cyc = [(0, 0), (1, 0), (1, 1), (0, 1)]
    P = [(nodeP[node(o)], nodeV[node(o)]) for o in cyc]
    V = 0.0
    G = 0.0
    for k in range(4):
        (pa, va), (pb, vb) = P[k], P[(k + 1) % 4]
        for (pc, vc), (p1, v1), (p2, v2) in (((CR, VR), (pa, va), (pb, vb)), ((CL, VL), (pb, vb), (pa, va))):
            S = 0.5 * _cross(p1 - pc, p2 - pc)
            V = V + (((pc + p1 + p2) / 3.0) * S).sum(0) / 3.0
            G = G + ((vc + v1 + v2) / 3.0)[:, None] * S[None]
    return G / V


def viscous_face_flux(grad, uf, Sd, mu, kcond):
    """F_v . S on faces: grad (dim+1, dim, faces...) of (u_1..u_dim, T), uf the
    face velocity (dim, faces...), Sd the area vectors (dim, faces...)."""
    dim = Sd.shape[0]
    gu = grad[:dim]  # gu[i, j] = du_i/dx_j
    div = sum(gu[i, i] for i in range(dim))
    tau = [[mu * (gu[i, j] + gu[j, i]) - (2.0 / 3.0 * mu * div if i == j else 0.0) for j in range(dim)]
           for i in range(dim)]
    mom = [sum(tau[i][j] * Sd[j] for j in range(dim)) for i in range(dim)]
    theta = [sum(uf[i] * tau[i][j] for i in range(dim)) + kcond * grad[dim, j] for j in range(dim)]
    energy = sum(theta[j] * Sd[j] for j in range(dim))
    return torch.stack([torch.zeros_like(energy)] + mom + [energy])


def viscous_residual(problem, pads, X_list, met):
    """Rv per block, (nvar, [nk,] nj, ni), from ghost-filled primitive pads."""
    dim, g = problem.dim, problem.gamma
    mu = problem.mu
    kcond = mu / ((g - 1.0) * problem.prandtl)
    S_list = [m[0] for m in met]
    padC = padded_centers(problem, X_list, S_list)
    out = []
    for b, qp in enumerate(pads):
        T = g * qp[-1] / qp[0]
        V = torch.cat([qp[1:-1], T[None]])  # (u.., T)
        nP = pseudo_nodes(padC[b], dim)
        nV = pseudo_nodes(V, dim)
        S, vol = met[b]
        nd = qp.ndim
        div = 0.0
        for d in range(dim):
            grad = face_gradients(padC[b], V, nP, nV, dim, d)
            ta = tensor_axis(nd, d)
            sl = [slice(None)] * nd
            for a in range(dim):
                sl[tensor_axis(nd, a)] = slice(2, -2) if a != d else slice(1, qp.shape[ta] - 1)
            # face velocity: mean of the two cells beside each face
            u = qp[1:-1][tuple(sl)]
            n = u.shape[ta] - 1
            uf = 0.5 * (u.narrow(ta, 0, n) + u.narrow(ta, 1, n))
            F = viscous_face_flux(grad, uf, S[d], mu, kcond)
            div = div + (F.narrow(ta, 1, n - 1) - F.narrow(ta, 0, n - 1))
        out.append(div / vol)
    return out


def viscous_rate(q, S, vol, mu, gamma, prandtl):
    """Viscous spectral-radius term of the time step per cell (reading):
    4 max(4/3, gamma/Pr) (mu/rho) sum_d |Sbar_d|^2 / Omega."""
    dim = q.shape[0] - 2
    acc = 0.0
    for d in range(dim):
        Sd = S[d]
        axS = tensor_axis(Sd.ndim, d)
        n = Sd.shape[axS] - 1
        Sbar = 0.5 * (Sd.narrow(axS, 0, n) + Sd.narrow(axS, 1, n))
        acc = acc + (Sbar * Sbar).sum(0)
    return 4.0 * max(4.0 / 3.0, gamma / prandtl) * mu / q[0] * acc / vol
