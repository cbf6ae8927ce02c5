"""Limiters and the kappa-form MUSCL face states.

Sec. 7.2 V4, eq. (flux): with Delta_{i+1/2} = q_{i+1} - q_i,

  q^L_{i+1/2} = q_i     + eps/4 [(1-kappa) Psi^+_{i-1/2} Delta_{i-1/2}
                                  + (1+kappa) Psi^-_{i+1/2} Delta_{i+1/2}]
  q^R_{i+1/2} = q_{i+1} - eps/4 [(1+kappa) Psi^+_{i+1/2} Delta_{i+1/2}
                                  + (1-kappa) Psi^-_{i+3/2} Delta_{i+3/2}]

applied to the primitive variables (Sec. 2: MUSCL "for the primitive
variables").  The paper does not define Psi^+-; reading (standard
upwind-biased ratios):

  Psi^+_{m} = Psi(Delta_{m+1} / Delta_{m}),  Psi^-_{m} = Psi(Delta_{m-1} / Delta_{m})

so every product Psi(a/b) b is evaluated in the slope form S(a, b), which is
also defined when b = 0 (the ratio is never formed):

  none       Psi = 1                        S(a, b) = b
  van Leer   Psi = (r + |r|)/(1 + |r|)      S(a, b) = (a|b| + |a|b)/(|a| + |b|), 0 if a = b = 0
  van Albada Psi = (r^2 + r)/(1 + r^2)      S(a, b) = ((b^2+e^2) a + (a^2+e^2) b)/(a^2 + b^2 + 2 e^2)

(van Albada with the usual regularisation e, per primitive variable.)

Limiter freezing (Sec. 8.2, the laminar NACA 0012 case: the limiter is frozen
late in a steady run so the residual keeps falling instead of oscillating; no
formula is printed).  Reading: for the symmetric limiters S(a, b) = S(b, a),
so one value per cell, direction and variable describes the limiter there,

  phi = S(a, b) / ((a + b) / 2)     (0 where a + b = 0, where S = 0 too),

the ratio of the limited slope to the central one, taken from the state at
the freeze.  Frozen, every product S(a, b) of the kappa-form becomes
phi (a + b) / 2 with the current differences a, b: the face states are
then linear in q, and at the freeze state they are unchanged.
"""
import torch


def _safe_div(num, den):
    ok = den != 0
    return torch.where(ok, num / torch.where(ok, den, torch.ones_like(den)), torch.zeros_like(num))


def slope(a, b, limiter, eps2=None):
    """S(a, b) = Psi(a / b) * b for the named limiter."""
    if limiter == "none":
        return b
    if limiter == "vanleer":
        return _safe_div(a * b.abs() + a.abs() * b, a.abs() + b.abs())
    if limiter == "vanalbada":
        e2 = torch.zeros_like(a) if eps2 is None else eps2
        return _safe_div((b * b + e2) * a + (a * a + e2) * b, a * a + b * b + 2.0 * e2)
    raise ValueError("unknown limiter %r" % limiter)


def psi(r, limiter):
    """The limiter as a function of the ratio (used only by the tests)."""
    if limiter == "none":
        return torch.ones_like(r)
    if limiter == "vanleer":
        return (r + r.abs()) / (1.0 + r.abs())
    if limiter == "vanalbada":
        return (r * r + r) / (1.0 + r * r)
    raise ValueError(limiter)


def frozen_factor(a, b, limiter, eps2=None):
    """phi = S(a, b) / ((a + b) / 2), 0 where a + b = 0."""
    return _safe_div(slope(a, b, limiter, eps2), 0.5 * (a + b))


def cell_differences(q, axis):
    """(Delta_{i-1/2}, Delta_{i+1/2}) of the cells -1 .. n of a padded array
    (n + 4 cells along ``axis``): the cells that touch the n + 1 faces."""
    m = q.shape[axis]
    D = q.narrow(axis, 1, m - 1) - q.narrow(axis, 0, m - 1)
    return D.narrow(axis, 0, m - 2), D.narrow(axis, 1, m - 2)


def face_states(q, axis, limiter, eps=1.0, kappa=-1.0, eps2=None, phi=None):
    """Left/right primitive states on the n+1 faces along ``axis`` of a
    padded array holding n + 4 cells along that axis (two ghost cells on each
    side).  Face f (0..n) lies between cells f-1 and f.

    ``phi``: frozen limiter factors of the cells -1 .. n (n + 2 along
    ``axis``), or None for the live limiter."""
    m = q.shape[axis]
    n = m - 4
    D = q.narrow(axis, 1, m - 1) - q.narrow(axis, 0, m - 1)  # D[p] = Delta between padded p, p+1
    Dm = D.narrow(axis, 0, n + 1)  # Delta_{i-1/2} for i = f-1
    D0 = D.narrow(axis, 1, n + 1)  # Delta_{i+1/2} = Delta_{f-1/2}
    Dp = D.narrow(axis, 2, n + 1)  # Delta_{i+3/2} = Delta_{f+1/2}
    e2 = eps2
    if phi is not None:
        # frozen: S(a, b) -> phi (a + b)/2 of the cell whose differences a, b are
        sL = phi.narrow(axis, 0, n + 1) * (0.5 * (D0 + Dm))
        sR = phi.narrow(axis, 1, n + 1) * (0.5 * (Dp + D0))
        qL = q.narrow(axis, 1, n + 1) + eps / 4.0 * ((1.0 - kappa) * sL + (1.0 + kappa) * sL)
        qR = q.narrow(axis, 2, n + 1) - eps / 4.0 * ((1.0 + kappa) * sR + (1.0 - kappa) * sR)
        return qL, qR
    # Psi^+_{i-1/2} Delta_{i-1/2} = S(Delta_{i+1/2}, Delta_{i-1/2});  Psi^-_{i+1/2} Delta_{i+1/2} = S(Delta_{i-1/2}, Delta_{i+1/2})
    qL = q.narrow(axis, 1, n + 1) + eps / 4.0 * ((1.0 - kappa) * slope(D0, Dm, limiter, e2)
                                                 + (1.0 + kappa) * slope(Dm, D0, limiter, e2))
    # Psi^+_{i+1/2} Delta_{i+1/2} = S(Delta_{i+3/2}, Delta_{i+1/2});  Psi^-_{i+3/2} Delta_{i+3/2} = S(Delta_{i+1/2}, Delta_{i+3/2})
    qR = q.narrow(axis, 2, n + 1) - eps / 4.0 * ((1.0 + kappa) * slope(Dp, D0, limiter, e2)
                                                 + (1.0 - kappa) * slope(D0, Dp, limiter, e2))
    return qL, qR
