"""Roe flux-difference splitting on a face with area vector S.

Sec. 2 names Roe's approximate Riemann solver (Roe 1981) as one of SENSEI's
inviscid fluxes without printing it; this is the textbook rotated form.
With A = |S| and unit normal n = S / A, for primitive states qL, qR:

  Roe averages (R = sqrt(rho_R / rho_L)):
    rho~ = R rho_L,  u~ = (u_L + R u_R)/(1 + R),  H~ = (H_L + R H_R)/(1 + R),
    c~^2 = (gamma - 1)(H~ - |u~|^2 / 2),  V~ = u~ . n
  wave strengths (d = right minus left, dV = du . n):
    a1 = (dp - rho~ c~ dV)/(2 c~^2),  a5 = (dp + rho~ c~ dV)/(2 c~^2),  a2 = drho - dp / c~^2
  eigenvalues l1 = V~ - c~, l2 = V~, l5 = V~ + c~
  dissipation
    D = |l1| a1 [1, u~ - c~ n, H~ - c~ V~]
      + |l2| (a2 [1, u~, |u~|^2/2] + rho~ [0, du - dV n, u~ . du - V~ dV])
      + |l5| a5 [1, u~ + c~ n, H~ + c~ V~]
  flux  F = A (F_n(qL) + F_n(qR) - D) / 2.

Entropy fix (not printed in the paper; reading): Harten's smoothing applied to
every eigenvalue, |l| -> (l^2 + delta^2)/(2 delta) where |l| < delta,
delta = efix * c~.  ``efix = 0`` disables it.  ``absfn`` replaces the
absolute value (the tests pass the identity to expose the Roe property).
"""
import torch

from .gas import normal_flux, total_enthalpy


def harten_abs(lam, delta):
    a = lam.abs()
    safe = torch.where(delta > 0, delta, torch.ones_like(delta))
    smooth = (lam * lam + delta * delta) / (2.0 * safe)
    return torch.where(a >= delta, a, smooth)


def roe_flux(qL, qR, S, gamma, efix=0.1, absfn=None):
    A = torch.sqrt((S * S).sum(0))
    n = S / A
    rhoL, velL, pL = qL[0], qL[1:-1], qL[-1]
    rhoR, velR, pR = qR[0], qR[1:-1], qR[-1]
    HL = total_enthalpy(qL, gamma)
    HR = total_enthalpy(qR, gamma)

    R = torch.sqrt(rhoR / rhoL)
    rho_t = R * rhoL
    u_t = (velL + R * velR) / (1.0 + R)
    H_t = (HL + R * HR) / (1.0 + R)
    q2_t = (u_t * u_t).sum(0)
    c2_t = (gamma - 1.0) * (H_t - 0.5 * q2_t)
    c_t = torch.sqrt(c2_t)
    V_t = (u_t * n).sum(0)

    drho = rhoR - rhoL
    dp = pR - pL
    du = velR - velL
    dV = (du * n).sum(0)

    a1 = (dp - rho_t * c_t * dV) / (2.0 * c2_t)
    a5 = (dp + rho_t * c_t * dV) / (2.0 * c2_t)
    a2 = drho - dp / c2_t

    l1 = V_t - c_t
    l2 = V_t
    l5 = V_t + c_t
    if absfn is None:
        delta = efix * c_t
        if efix > 0:
            absfn = lambda lam: harten_abs(lam, delta)
        else:
            absfn = torch.abs
    m1, m2, m5 = absfn(l1), absfn(l2), absfn(l5)

    one = torch.ones_like(rho_t)
    r1 = torch.cat([one[None], u_t - c_t * n, (H_t - c_t * V_t)[None]])
    r5 = torch.cat([one[None], u_t + c_t * n, (H_t + c_t * V_t)[None]])
    r2 = torch.cat([one[None], u_t, (0.5 * q2_t)[None]])
    shear = torch.cat([torch.zeros_like(rho_t)[None], du - dV * n, ((u_t * du).sum(0) - V_t * dV)[None]])
    D = m1 * a1 * r1 + m2 * (a2 * r2 + rho_t * shear) + m5 * a5 * r5

    FL = normal_flux(qL, n, gamma)
    FR = normal_flux(qR, n, gamma)
    return A * (0.5 * (FL + FR) - 0.5 * D)
