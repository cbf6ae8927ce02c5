"""Residual, time step, Runge-Kutta update and wall-pressure objective.

* Residual: finite-volume form of eq. (1), Sec. 2, inviscid part with no
  source: for every cell, R = (1/Omega) sum over its faces of the outward
  numerical flux times area, so that dQ/dt = -R.  Faces are visited one index
  direction at a time: MUSCL face states (muscl.face_states) and the scheme's
  face flux (roe.roe_flux by default, or a flux-vector splitting of fvs) on
  every face of the direction, then the flux difference.
* Wall faces: Sec. 7.2 V7 overwrites the Riemann flux on wall faces after the
  boundary enforcement.  Reading: F = (0, p_w S, 0) with the wall pressure
  extrapolated linearly in index space, p_w = 1.5 p_0 - 0.5 p_1 (p_0 the cell
  adjacent to the wall, p_1 the next one in).
* Farfield faces: V7 overwrites those too.  Reading: the face flux is the
  exact normal flux of the characteristic boundary state q_b (oracle/bc.py)
  that the farfield ghost cells hold, F = F(q_b) . S.
* Time step: the paper does not state it.  Reading: a global step
  dt = CFL * min over all cells of Omega / lambda, with
  lambda = sum_d (|u . Sbar_d| + c |Sbar_d|), Sbar_d the mean of the cell's
  two area vectors in direction d, evaluated once per step from Q^n.
* Runge-Kutta: Sec. 2, the explicit M-step scheme of Jameson, Schmidt and
  Turkel: Q^(k) = Q^(0) - alpha_k dt R(Q^(k-1)), alpha_k = 1/(M - k + 1).
  Optionally (rk_scheme "classic4", not in the paper) the classical
  fourth-order Runge-Kutta method written from its textbook definition:
  k_i = -R(Y_i) with Y_1 = Q^n, Y_2 = Q^n + dt/2 k_1, Y_3 = Q^n + dt/2 k_2,
  Y_4 = Q^n + dt k_3, and Q^(n+1) = Q^n + dt/6 (k_1 + 2 k_2 + 2 k_3 + k_4).
* Objective: J = sum over slip-wall faces of p_w |S| (integrated wall pressure).
* Laminar Navier-Stokes (viscosity > 0): R = R_inviscid - Rv with the
  viscous residual of oracle/viscous.py; no-slip walls take the inviscid wall
  override too; the time step adds the viscous rate of oracle/viscous.py to
  lambda.
"""
from __future__ import annotations

import torch

from . import fvs, gas, metrics as metrics_mod, muscl, roe, viscous
from .ghosts import boundary_state, face_area_slab, fill_ghosts, interior_layer, tangential_axes, tensor_axis

F64 = torch.float64


class _Patch:
    def __init__(self, p, index):
        self.block, self.face, self.lo, self.hi, self.kind = p.block, p.face, list(p.lo), list(p.hi), p.kind
        self.index = index
        self.params = list(p.params) if p.params is not None else None


class Problem:
    """Blocks, topology and scheme of a ``synth.Case`` as oracle tensors.

    ``nodes`` and the inflow parameters are leaf tensors so gradients with
    respect to them can be taken with torch.autograd."""

    def __init__(self, case, requires_grad=False):
        self.case = case
        self.dim = case.dim
        self.nvar = case.dim + 2
        sch = case.scheme
        self.gamma = sch.gamma
        self.limiter = sch.limiter
        self.eps = sch.muscl_eps
        self.kappa = sch.muscl_kappa
        self.efix = sch.efix
        self.flux = getattr(sch, "flux", "roe")
        self.stages = sch.rk_stages
        self.rk_scheme = getattr(sch, "rk_scheme", "mstage")
        self.cfl = sch.cfl
        self.dt_fixed = sch.dt_fixed
        self.local_dt = getattr(sch, "local_dt", False)
        self.frozen = None  # per block, per direction: frozen limiter factors (muscl.frozen_factor)
        self.mu = float(getattr(sch, "viscosity", 0.0))
        self.prandtl = float(getattr(sch, "prandtl", 0.72))
        le = sch.lim_eps if sch.lim_eps is not None else [0.0] * self.nvar
        self.lim_eps2 = torch.tensor([e * e for e in le], dtype=F64)
        self.nodes = [torch.tensor(b.nodes, dtype=F64, requires_grad=requires_grad) for b in case.blocks]
        self.conns = case.conns
        self.bcs = []
        self.bc_params = []
        for p in case.bcs:
            self.bcs.append(_Patch(p, len(self.bc_params) if p.kind == "sup_inflow" else -1))
            if p.kind == "sup_inflow":
                self.bc_params.append(torch.tensor(p.params, dtype=F64, requires_grad=requires_grad))

    # -- grid ---------------------------------------------------------------
    def metrics(self):
        return [metrics_mod.metrics(X) for X in self.nodes]

    # -- state conversions --------------------------------------------------
    def initial_state(self):
        return [gas.cons_from_prim(torch.tensor(q, dtype=F64), self.gamma) for q in self.case.prims]

    # -- residual -----------------------------------------------------------
    def block_residual_padded(self, qpad, S, vol, walls=(), phi=None):
        """Residual of one block from a padded primitive array (ghosts given).

        ``walls``: boundary patches of the block whose face flux is overwritten
        (slip walls and farfield faces), or (face, lo, hi) triples of slip walls.
        ``phi``: frozen limiter factors of the block per direction, or None."""
        dim = self.dim
        nd = qpad.ndim
        eps2 = self.lim_eps2.reshape([-1] + [1] * (nd - 1))
        div = 0.0
        for d in range(dim):
            ax = tensor_axis(nd, d)
            # interior range in the other directions, full padded range along d
            sl = [slice(None)] * nd
            for a in range(dim):
                if a != d:
                    sl[tensor_axis(nd, a)] = slice(2, -2)
            qd = qpad[tuple(sl)]
            qL, qR = muscl.face_states(qd, ax, self.limiter, self.eps, self.kappa, eps2,
                                       None if phi is None else phi[d])
            F = self.face_flux(qL, qR, S[d])
            for w in walls:
                face, lo, hi = (w.face, w.lo, w.hi) if isinstance(w, _Patch) else w
                if face // 2 != d:
                    continue
                if isinstance(w, _Patch) and w.kind == "farfield":
                    F = self._farfield_override(F, qpad, S, w)
                else:
                    F = self._wall_override(F, qpad, S[d], face, lo, hi)
            n = F.shape[ax] - 1
            div = div + (F.narrow(ax, 1, n) - F.narrow(ax, 0, n))
        return div / vol

    def face_flux(self, qL, qR, S):
        """Inviscid face flux of the scheme: Roe (default), van Leer or
        Steger-Warming flux-vector splitting."""
        if self.flux == "roe":
            return roe.roe_flux(qL, qR, S, self.gamma, self.efix)
        if self.flux == "vanleer_fvs":
            return fvs.van_leer_flux(qL, qR, S, self.gamma)
        if self.flux == "steger_warming":
            return fvs.steger_warming_flux(qL, qR, S, self.gamma)
        raise ValueError("unknown flux %s" % self.flux)

    def _wall_override(self, F, qpad, Sd, face, lo, hi):
        dim, nd = self.dim, F.ndim
        ax = tensor_axis(nd, face // 2)
        q = qpad[tuple([slice(None)] + [slice(2, -2)] * dim)]
        p0 = interior_layer(q, dim, face, 0, lo, hi)[-1]
        p1 = interior_layer(q, dim, face, 1, lo, hi)[-1]
        pw = 1.5 * p0 - 0.5 * p1
        sl = [slice(None)] * nd
        sl[ax] = 0 if face % 2 == 0 else F.shape[ax] - 1
        for t, a in enumerate(tangential_axes(dim, face)):
            sl[tensor_axis(nd, a)] = slice(lo[t], hi[t])
        Sf = Sd[tuple(sl)]
        if dim == 3:
            Sf = Sf.permute(0, 2, 1)  # to (dim, t1, t2) like pw
        mom = pw[None] * Sf
        zero = torch.zeros_like(pw)[None]
        Fw = torch.cat([zero, mom, zero])
        if dim == 3:
            Fw = Fw.permute(0, 2, 1)
        F = F.clone()
        F[tuple(sl)] = Fw
        return F

    def _farfield_override(self, F, qpad, S, p):
        dim, nd = self.dim, F.ndim
        ax = tensor_axis(nd, p.face // 2)
        q = qpad[tuple([slice(None)] + [slice(2, -2)] * dim)]
        qb = boundary_state(self, p, q, S)
        Sf = face_area_slab(S[p.face // 2], dim, p.face, p.lo, p.hi)
        area = torch.sqrt((Sf * Sf).sum(0))
        Fb = gas.normal_flux(qb, Sf / area, self.gamma) * area
        sl = [slice(None)] * nd
        sl[ax] = 0 if p.face % 2 == 0 else F.shape[ax] - 1
        for t, a in enumerate(tangential_axes(dim, p.face)):
            sl[tensor_axis(nd, a)] = slice(p.lo[t], p.hi[t])
        if dim == 3:
            Fb = Fb.permute(0, 2, 1)
        F = F.clone()
        F[tuple(sl)] = Fb
        return F

    def walls_of(self, b):
        """Patches of block b whose face flux is overwritten: slip walls and farfield."""
        return [p for p in self.bcs if p.block == b and p.kind in ("slip_wall", "noslip_wall", "farfield")]

    def residual(self, Q_list, met=None):
        met = self.metrics() if met is None else met
        q_list = [gas.prim_from_cons(Q, self.gamma) for Q in Q_list]
        S_list = [m[0] for m in met]
        pads = fill_ghosts(self, q_list, S_list)
        R = [self.block_residual_padded(pads[b], met[b][0], met[b][1], self.walls_of(b),
                                        None if self.frozen is None else self.frozen[b])
             for b in range(len(Q_list))]
        if self.mu > 0.0:
            Rv = viscous.viscous_residual(self, pads, self.nodes, met)
            R = [r - rv for r, rv in zip(R, Rv)]
        return R

    # -- limiter freezing ---------------------------------------------------
    def freeze_limiter(self, Q_list, met=None):
        """Freeze the limiter at the state Q_list (muscl.frozen_factor of every
        cell -1 .. n per direction, from the ghost-filled primitives); later
        residuals use the frozen factors until unfreeze_limiter()."""
        if self.limiter == "none":
            raise ValueError("no limiter to freeze")
        met = self.metrics() if met is None else met
        q_list = [gas.prim_from_cons(Q, self.gamma) for Q in Q_list]
        pads = fill_ghosts(self, q_list, [m[0] for m in met])
        dim = self.dim
        self.frozen = []
        for qpad in pads:
            nd = qpad.ndim
            eps2 = self.lim_eps2.reshape([-1] + [1] * (nd - 1))
            per_dir = []
            for d in range(dim):
                sl = [slice(None)] * nd
                for a in range(dim):
                    if a != d:
                        sl[tensor_axis(nd, a)] = slice(2, -2)
                Dm, Dp = muscl.cell_differences(qpad[tuple(sl)], tensor_axis(nd, d))
                per_dir.append(muscl.frozen_factor(Dp, Dm, self.limiter, eps2))
            self.frozen.append(per_dir)

    def unfreeze_limiter(self):
        self.frozen = None

    # -- time step ----------------------------------------------------------
    def cell_dt(self, Q, S, vol):
        """Omega / lambda per cell."""
        q = gas.prim_from_cons(Q, self.gamma)
        c = gas.sound_speed(q, self.gamma)
        vel = q[1:-1]
        lam = 0.0
        for d in range(self.dim):
            Sd = S[d]
            n = Sd.shape[tensor_axis(Sd.ndim, d)] - 1
            axS = tensor_axis(Sd.ndim, d)
            Sbar = 0.5 * (Sd.narrow(axS, 0, n) + Sd.narrow(axS, 1, n))
            lam = lam + (vel * Sbar).sum(0).abs() + c * torch.sqrt((Sbar * Sbar).sum(0))
        if self.mu > 0.0:
            lam = lam + viscous.viscous_rate(q, S, vol, self.mu, self.gamma, self.prandtl)
        return vol / lam

    def time_step(self, Q_list, met=None):
        if self.dt_fixed is not None:
            return torch.tensor(self.dt_fixed, dtype=F64)
        met = self.metrics() if met is None else met
        m = min(self.cell_dt(Q, met[b][0], met[b][1]).min() for b, Q in enumerate(Q_list))
        return self.cfl * m

    def local_steps(self, Q_list, met=None):
        """Local time stepping (steady-state acceleration): every cell advances
        with its own dt_i = CFL * Omega_i / lambda_i from Q^n."""
        met = self.metrics() if met is None else met
        return [self.cfl * self.cell_dt(Q, met[b][0], met[b][1]) for b, Q in enumerate(Q_list)]

    # -- Runge-Kutta --------------------------------------------------------
    def rk_step(self, Q_list, met=None, dt=None, residual_fn=None):
        """One M-stage step.  Returns the new state and the step: the global
        dt, or with local stepping the smallest cell step."""
        met = self.metrics() if met is None else met
        if self.local_dt and dt is None:
            dts = self.local_steps(Q_list, met)
            dt = min(d.min() for d in dts)
        else:
            dt = self.time_step(Q_list, met) if dt is None else dt
            dts = [dt] * len(Q_list)
        res = (lambda Qs: self.residual(Qs, met)) if residual_fn is None else residual_fn
        if self.rk_scheme == "classic4":
            return self._classic4(Q_list, dts, res), dt
        M = self.stages
        Q0 = Q_list
        Qk = Q_list
        for k in range(1, M + 1):
            alpha = 1.0 / (M - k + 1)
            R = res(Qk)
            Qk = [Q0[b] - alpha * dts[b] * R[b] for b in range(len(Q0))]
        return Qk, dt

    def _classic4(self, Q0, dts, res):
        nb = range(len(Q0))
        k1 = [-r for r in res(Q0)]
        k2 = [-r for r in res([Q0[b] + 0.5 * dts[b] * k1[b] for b in nb])]
        k3 = [-r for r in res([Q0[b] + 0.5 * dts[b] * k2[b] for b in nb])]
        k4 = [-r for r in res([Q0[b] + dts[b] * k3[b] for b in nb])]
        return [Q0[b] + dts[b] / 6.0 * (k1[b] + 2.0 * k2[b] + 2.0 * k3[b] + k4[b]) for b in nb]

    def residual_norms(self, Q_list, met=None):
        """Root-mean-square residual per conservative variable over all cells
        (the convergence monitor of steady runs)."""
        R = self.residual(Q_list, met)
        n = sum(r[0].numel() for r in R)
        ss = sum((r.reshape(self.nvar, -1) ** 2).sum(1) for r in R)
        return torch.sqrt(ss / n)

    def run(self, Q_list, steps, met=None):
        met = self.metrics() if met is None else met
        dts = []
        for _ in range(steps):
            Q_list, dt = self.rk_step(Q_list, met)
            dts.append(dt)
        return Q_list, dts

    # -- objective ----------------------------------------------------------
    def wall_pressure_integral(self, Q_list, met=None):
        met = self.metrics() if met is None else met
        J = torch.zeros((), dtype=F64)
        for p in self.bcs:
            if p.kind != "slip_wall":
                continue
            q = gas.prim_from_cons(Q_list[p.block], self.gamma)
            p0 = interior_layer(q, self.dim, p.face, 0, p.lo, p.hi)[-1]
            p1 = interior_layer(q, self.dim, p.face, 1, p.lo, p.hi)[-1]
            pw = 1.5 * p0 - 0.5 * p1
            S = met[p.block][0][p.face // 2]
            Sf = face_area_slab(S, self.dim, p.face, p.lo, p.hi)
            J = J + (pw * torch.sqrt((Sf * Sf).sum(0))).sum()
        return J
