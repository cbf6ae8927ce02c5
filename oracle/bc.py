"""Characteristic boundary states: farfield, subsonic inflow, subsonic outflow.

Sec. 2 lists SENSEI's boundary types (including farfield and subsonic
inflow/outflow) and Sec. 7.2 V7 overwrites the face flux on wall and farfield
faces; the paper prints no formulas.  Readings (textbook forms), with q_i the
primitive state of the interior cell next to the face and n the unit normal
pointing out of the domain:

* farfield (Riemann invariants): V = u . n, c = sqrt(gamma p / rho).
  Supersonic outflow (V_i >= c_i): q_b = q_i.  Supersonic inflow
  (V_inf <= -c_inf): q_b = q_inf.  Otherwise
      R+ = V_i + 2 c_i / (gamma - 1),   R- = V_inf - 2 c_inf / (gamma - 1),
      V_b = (R+ + R-) / 2,              c_b = (gamma - 1)(R+ - R-) / 4,
  and the tangential velocity and entropy s = p / rho^gamma come from q_i
  where V_b >= 0 (outflow), from q_inf where V_b < 0 (inflow):
      rho_b = (c_b^2 / (gamma s))^(1/(gamma-1)),  p_b = rho_b c_b^2 / gamma,
      u_b = u_side - (u_side . n) n + V_b n.
  The farfield face flux is the normal flux of q_b (the V7 overwrite).
* subsonic inflow, parameters (p0, rho0, d): stagnation pressure and density
  and the unit inflow direction d (into the domain).  The static pressure is
  extrapolated, p_b = min(p_i, p0), and the isentropic relations give
      rho_b = rho0 (p_b / p0)^(1/gamma),
      |u_b|^2 = 2 gamma / (gamma - 1) (p0 / rho0 - p_b / rho_b),  u_b = |u_b| d.
* subsonic outflow, parameter p_back: q_b = (rho_i, u_i, p_back) while
  V_i < c_i; q_b = q_i when the outflow is supersonic.

Both ghost layers hold q_b.  TEST INFRASTRUCTURE ONLY (part of the oracle).
"""
import torch


def _sound(q, gamma):
    return torch.sqrt(gamma * q[-1] / q[0])


def farfield_state(q_i, n_out, q_inf, gamma):
    """q_i (nvar, ...), n_out (dim, ...) unit outward normal, q_inf (nvar,)."""
    shape = [-1] + [1] * (q_i.ndim - 1)
    q_f = q_inf.reshape(shape).expand_as(q_i)
    ci, cf = _sound(q_i, gamma), _sound(q_f, gamma)
    Vi = (q_i[1:-1] * n_out).sum(0)
    Vf = (q_f[1:-1] * n_out).sum(0)
    Rp = Vi + 2.0 * ci / (gamma - 1.0)
    Rm = Vf - 2.0 * cf / (gamma - 1.0)
    Vb = 0.5 * (Rp + Rm)
    cb = 0.25 * (gamma - 1.0) * (Rp - Rm)
    out = Vb >= 0.0
    side = torch.where(out, q_i, q_f)
    s = side[-1] / side[0] ** gamma
    rho_b = (cb * cb / (gamma * s)) ** (1.0 / (gamma - 1.0))
    p_b = rho_b * cb * cb / gamma
    us = side[1:-1]
    u_b = us - (us * n_out).sum(0) * n_out + Vb * n_out
    qb = torch.cat([rho_b[None], u_b, p_b[None]])
    qb = torch.where(Vi >= ci, q_i, qb)
    return torch.where(Vf <= -cf, q_f, qb)


def subsonic_inflow_state(q_i, params, gamma):
    """params = (p0, rho0, d_1 .. d_dim) with d the inflow direction (normalised here)."""
    p0, rho0 = params[0], params[1]
    d = params[2:2 + q_i.shape[0] - 2]
    d = d / torch.sqrt((d * d).sum())
    pb = torch.minimum(q_i[-1], p0.expand_as(q_i[-1]))
    rho_b = rho0 * (pb / p0) ** (1.0 / gamma)
    speed = torch.sqrt(torch.clamp(2.0 * gamma / (gamma - 1.0) * (p0 / rho0 - pb / rho_b), min=0.0))
    u_b = speed * d.reshape([-1] + [1] * (q_i.ndim - 1))
    return torch.cat([rho_b[None], u_b, pb[None]])


def subsonic_outflow_state(q_i, n_out, p_back, gamma):
    ci = _sound(q_i, gamma)
    Vi = (q_i[1:-1] * n_out).sum(0)
    qb = torch.cat([q_i[:-1], p_back.expand_as(q_i[-1])[None]])
    return torch.where(Vi >= ci, q_i, qb)
