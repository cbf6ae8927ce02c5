"""Flux-vector splittings on a face with area vector S.

Sec. 2 lists van Leer's and Steger and Warming's flux-vector splittings among
SENSEI's inviscid fluxes (beside Roe's flux-difference splitting) without
printing them; these are the textbook forms.  With A = |S|, n = S / A and the
normal velocity V = u . n, the face flux is

    F = A (F+(qL) + F-(qR)).

Steger-Warming: the normal Euler flux is homogeneous of degree one in the
conservative state, F_n(Q) = A_n(Q) Q, and A_n = R diag(l) R^-1 with
eigenvalues l1 = V - c, l2 = V (repeated), l3 = V + c.  Splitting every
eigenvalue into l+ = (l + |l|)/2 and l- = (l - |l|)/2 gives F+- = R diag(l+-)
R^-1 Q, whose closed form (each l below is its + or - part) is

    F+- = rho / (2 gamma) [ a,
                            a u + c (l3 - l1) n,
                            a |u|^2 / 2 + c V (l3 - l1) + c^2 (l1 + l3) / (gamma - 1) ],
    a = 2 (gamma - 1) l2 + l1 + l3.

van Leer: with the normal Mach number M = V / c, F+ = F_n, F- = 0 for M >= 1
(mirror for M <= -1); for |M| < 1 the mass flux f+- = +- rho c (M +- 1)^2 / 4
and

    F+- = f+- [ 1,
                u + n (-V +- 2 c) / gamma,
                (|u|^2 - V^2) / 2 + ((gamma - 1) V +- 2 c)^2 / (2 (gamma^2 - 1)) ].

TEST INFRASTRUCTURE ONLY (part of the oracle).
"""
import torch

from .gas import normal_flux, sound_speed


def _frame(q, S):
    A = torch.sqrt((S * S).sum(0))
    n = S / A
    vel = q[1:-1]
    V = (vel * n).sum(0)
    return A, n, V


def steger_warming_part(q, n, gamma, sign):
    """F+ (sign = +1) or F- (sign = -1) of the Steger-Warming splitting for the
    primitive state q and unit normal n (flux per unit area)."""
    rho, vel, p = q[0], q[1:-1], q[-1]
    c = sound_speed(q, gamma)
    V = (vel * n).sum(0)
    lam = [V - c, V, V + c]
    lp = [0.5 * (l + sign * l.abs()) for l in lam]
    l1, l2, l3 = lp
    a = 2.0 * (gamma - 1.0) * l2 + l1 + l3
    k = rho / (2.0 * gamma)
    q2 = (vel * vel).sum(0)
    mass = k * a
    mom = k * (a * vel + c * (l3 - l1) * n)
    en = k * (a * 0.5 * q2 + c * V * (l3 - l1) + c * c * (l1 + l3) / (gamma - 1.0))
    return torch.cat([mass[None], mom, en[None]])


def van_leer_part(q, n, gamma, sign):
    """F+ (sign = +1) or F- (sign = -1) of van Leer's splitting (per unit area)."""
    rho, vel, p = q[0], q[1:-1], q[-1]
    c = sound_speed(q, gamma)
    V = (vel * n).sum(0)
    M = V / c
    q2 = (vel * vel).sum(0)
    f = sign * rho * c * (M + sign) ** 2 / 4.0
    mass = f
    mom = f * (vel + n * (-V + sign * 2.0 * c) / gamma)
    en = f * (0.5 * (q2 - V * V) + ((gamma - 1.0) * V + sign * 2.0 * c) ** 2 / (2.0 * (gamma * gamma - 1.0)))
    sub = torch.cat([mass[None], mom, en[None]])
    full = normal_flux(q, n, gamma)
    supersonic_own = (M >= 1.0) if sign > 0 else (M <= -1.0)
    supersonic_other = (M <= -1.0) if sign > 0 else (M >= 1.0)
    out = torch.where(supersonic_own, full, sub)
    return torch.where(supersonic_other, torch.zeros_like(out), out)


def steger_warming_flux(qL, qR, S, gamma):
    A, n, _ = _frame(qL, S)
    return A * (steger_warming_part(qL, n, gamma, 1.0) + steger_warming_part(qR, n, gamma, -1.0))


def van_leer_flux(qL, qR, S, gamma):
    A, n, _ = _frame(qL, S)
    return A * (van_leer_part(qL, n, gamma, 1.0) + van_leer_part(qR, n, gamma, -1.0))
