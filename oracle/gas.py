"""Ideal-gas variables and the inviscid normal flux.

Sec. 2 (SENSEI), eq. (2): conserved Q = (rho, rho u, rho v, rho w, rho e_t) and
inviscid normal flux F_n = (rho V_n, rho u V_n + n_x p, ..., rho h_t V_n) with
V_n = n . u for a unit face normal n.  Perfect gas: p = (gamma-1)(rho e_t -
rho |u|^2 / 2), h_t = e_t + p / rho.

Tensors have the variable index first: (nvar, ...), nvar = dim + 2.
"""
import torch


def cons_from_prim(q, gamma):
    rho, vel, p = q[0], q[1:-1], q[-1]
    mom = rho * vel
    rhoE = p / (gamma - 1.0) + 0.5 * rho * (vel * vel).sum(0)
    return torch.cat([rho[None], mom, rhoE[None]])


def prim_from_cons(Q, gamma):
    rho, mom, rhoE = Q[0], Q[1:-1], Q[-1]
    vel = mom / rho
    p = (gamma - 1.0) * (rhoE - 0.5 * rho * (vel * vel).sum(0))
    return torch.cat([rho[None], vel, p[None]])


def total_enthalpy(q, gamma):
    rho, vel, p = q[0], q[1:-1], q[-1]
    return gamma / (gamma - 1.0) * p / rho + 0.5 * (vel * vel).sum(0)


def sound_speed(q, gamma):
    return torch.sqrt(gamma * q[-1] / q[0])


def normal_flux(q, n, gamma):
    """Inviscid flux through a face with unit normal ``n`` (dim, ...) for the
    primitive state ``q``; eq. (2) of Sec. 2."""
    rho, vel, p = q[0], q[1:-1], q[-1]
    vn = (vel * n).sum(0)
    H = total_enthalpy(q, gamma)
    return torch.cat([(rho * vn)[None], rho * vel * vn + p * n, (rho * H * vn)[None]])
