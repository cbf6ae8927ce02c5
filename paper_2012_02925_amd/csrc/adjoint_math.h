// Reverse-mode derivatives (vector-Jacobian products) of the per-face and
// per-cell arithmetic in device_math.h, written by hand.
#pragma once

#include "device_math.h"

namespace cfd {

// Slope S(a, b) and its partial derivatives dS/da, dS/db (symmetric limiters).
// At a vanishing denominator the slope is 0 with zero partials, as the
// forward path returns 0 there.
template <int LIM>
__device__ __forceinline__ void slope_partials(double a, double b, double e2, double& s, double& sa, double& sb) {
  if constexpr (LIM == LIM_VANLEER) {
    const double aa = fabs(a), ab = fabs(b);
    const double sga = a > 0.0 ? 1.0 : (a < 0.0 ? -1.0 : 0.0);
    const double sgb = b > 0.0 ? 1.0 : (b < 0.0 ? -1.0 : 0.0);
    const double den = aa + ab;
    const double num = a * ab + aa * b;
    if (den > SLOPE_TINY) {
      const double id = rcp(den);
      s = num * id;
      sa = ((ab + sga * b) - s * sga) * id;
      sb = ((a * sgb + aa) - s * sgb) * id;
    } else {
      s = sa = sb = 0.0;
    }
  } else {
    const double a2 = a * a, b2 = b * b;
    const double den = a2 + b2 + 2.0 * e2;
    const double num = (b2 + e2) * a + (a2 + e2) * b;
    if (den > SLOPE_TINY) {
      const double id = rcp(den);
      s = num * id;
      sa = ((b2 + e2) + 2.0 * a * b - s * 2.0 * a) * id;
      sb = (2.0 * a * b + (a2 + e2) - s * 2.0 * b) * id;
    } else {
      s = sa = sb = 0.0;
    }
  }
}

// Per-cell slope cotangent split: given the cotangents of the high-face slope
// (spb) and the low-face slope (smb) of a cell, return the cotangents of the
// forward difference dp = q_{i+1} - q_i (gp) and backward difference
// dm = q_i - q_{i-1} (hm).  Symmetric limiters: sp = sm = S(dp, dm).
template <int LIM>
__device__ __forceinline__ void slope_vjp(double dm, double dp, double e2, double kap, double spb, double smb,
                                          double& gp, double& hm) {
  if constexpr (LIM == LIM_NONE) {
    // sp = ((1-k) dm + (1+k) dp)/2, sm = ((1+k) dm + (1-k) dp)/2
    gp = 0.5 * ((1.0 + kap) * spb + (1.0 - kap) * smb);
    hm = 0.5 * ((1.0 - kap) * spb + (1.0 + kap) * smb);
  } else {
    double s, sa, sb;
    slope_partials<LIM>(dp, dm, e2, s, sa, sb);
    const double tb = spb + smb;
    gp = tb * sa;
    hm = tb * sb;
  }
}

__device__ __forceinline__ void habs_vjp(double l, double delta, double inv2d, double efix, double mbar, double& lbar,
                                         double& ctbar) {
  const double a = fabs(l);
  if (a >= delta) {
    lbar += mbar * (l > 0.0 ? 1.0 : (l < 0.0 ? -1.0 : 0.0));
  } else {
    // m = (l^2 + delta^2) / (2 delta), delta = efix c~
    lbar += mbar * 2.0 * l * inv2d;
    ctbar += mbar * efix * (delta * delta - l * l) * 2.0 * inv2d * inv2d;
  }
}

// Roe flux (roe_flux in device_math.h) and its vector-Jacobian product:
// given Fb = dJ/dF, accumulate dJ/dqL into qLb, dJ/dqR into qRb and dJ/dS
// into Sb.  F receives the flux itself.
template <int DIM>
__device__ __forceinline__ void roe_flux_vjp(const double* qL, const double* qR, const double* S, const Gas& g,
                                             double efix, double half_inv_efix, const double* Fb, double* F,
                                             double* qLb, double* qRb, double* Sb) {
  constexpr int NV = DIM + 2;
  // ---------------- forward (same operations as roe_flux) ----------------
  double A2 = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) A2 += S[d] * S[d];
  const double iA = rsq(A2);
  const double A = A2 * iA;
  double n[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) n[d] = S[d] * iA;
  const double rL = qL[0], rR = qR[0];
  const double pL = qL[NV - 1], pR = qR[NV - 1];
  const double* uL = qL + 1;
  const double* uR = qR + 1;
  double vnL = 0.0, vnR = 0.0, keL = 0.0, keR = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    vnL += uL[d] * n[d];
    vnR += uR[d] * n[d];
    keL += uL[d] * uL[d];
    keR += uR[d] * uR[d];
  }
  const double irL = rcp(rL), irR = rcp(rR);
  const double HL = g.g_gm1 * pL * irL + 0.5 * keL;
  const double HR = g.g_gm1 * pR * irR + 0.5 * keR;
  const double ratio = rR * irL;
  const double R = ratio * rsq(ratio);
  const double iR1 = rcp(1.0 + R);
  const double rt = R * rL;
  double ut[DIM];
  double q2t = 0.0, Vt = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    ut[d] = (uL[d] + R * uR[d]) * iR1;
    q2t += ut[d] * ut[d];
    Vt += ut[d] * n[d];
  }
  const double Ht = (HL + R * HR) * iR1;
  const double c2t = g.gm1 * (Ht - 0.5 * q2t);
  const double ict = rsq(c2t);
  const double ct = c2t * ict;
  const double ic2 = ict * ict;
  const double drho = rR - rL;
  const double dp = pR - pL;
  double du[DIM];
  double dV = 0.0, udu = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    du[d] = uR[d] - uL[d];
    dV += du[d] * n[d];
    udu += ut[d] * du[d];
  }
  const double rcdV = rt * ct * dV;
  const double a1 = 0.5 * (dp - rcdV) * ic2;
  const double a5 = 0.5 * (dp + rcdV) * ic2;
  const double a2 = drho - dp * ic2;
  const double l1 = Vt - ct, l2 = Vt, l5 = Vt + ct;
  double m1, m2, m5, delta = 0.0, inv2d = 0.0;
  if (efix > 0.0) {
    delta = efix * ct;
    inv2d = half_inv_efix * ict;
    m1 = habs(l1, delta, inv2d);
    m2 = habs(l2, delta, inv2d);
    m5 = habs(l5, delta, inv2d);
  } else {
    m1 = fabs(l1);
    m2 = fabs(l2);
    m5 = fabs(l5);
  }
  const double w1 = m1 * a1, w5 = m5 * a5, w2 = m2 * a2, ws = m2 * rt;
  const double hA = 0.5 * A;
  double Dm[DIM];
  const double B0 = rL * vnL + rR * vnR - (w1 + w2 + w5);
  double Bm[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    Dm[d] = w1 * (ut[d] - ct * n[d]) + w2 * ut[d] + ws * (du[d] - dV * n[d]) + w5 * (ut[d] + ct * n[d]);
    Bm[d] = rL * uL[d] * vnL + pL * n[d] + rR * uR[d] * vnR + pR * n[d] - Dm[d];
  }
  const double De = w1 * (Ht - ct * Vt) + w2 * 0.5 * q2t + ws * (udu - Vt * dV) + w5 * (Ht + ct * Vt);
  const double Be = rL * HL * vnL + rR * HR * vnR - De;
  F[0] = hA * B0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) F[1 + d] = hA * Bm[d];
  F[NV - 1] = hA * Be;

  // ---------------- reverse ----------------
  double rLb = 0.0, rRb = 0.0, pLb = 0.0, pRb = 0.0, uLb[DIM], uRb[DIM], nb[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) uLb[d] = uRb[d] = nb[d] = 0.0;
  double hAb = Fb[0] * B0 + Fb[NV - 1] * Be;
#pragma unroll
  for (int d = 0; d < DIM; ++d) hAb += Fb[1 + d] * Bm[d];
  const double G0 = hA * Fb[0], Ge = hA * Fb[NV - 1];
  double vnLb = 0.0, vnRb = 0.0, w1b = 0.0, w2b = 0.0, w5b = 0.0, wsb = 0.0;
  double utb[DIM], dub[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) utb[d] = dub[d] = 0.0;
  double ctb = 0.0, dVb = 0.0, Htb = 0.0, Vtb = 0.0, q2tb = 0.0, udub = 0.0, HLb = 0.0, HRb = 0.0;
  // B0
  rLb += G0 * vnL;
  vnLb += G0 * rL;
  rRb += G0 * vnR;
  vnRb += G0 * rR;
  w1b -= G0;
  w2b -= G0;
  w5b -= G0;
  // Bm, Dm
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double Gm = hA * Fb[1 + d];
    rLb += Gm * uL[d] * vnL;
    uLb[d] += Gm * rL * vnL;
    vnLb += Gm * rL * uL[d];
    rRb += Gm * uR[d] * vnR;
    uRb[d] += Gm * rR * vnR;
    vnRb += Gm * rR * uR[d];
    pLb += Gm * n[d];
    pRb += Gm * n[d];
    nb[d] += Gm * (pL + pR);
    const double Dmb = -Gm;
    w1b += Dmb * (ut[d] - ct * n[d]);
    w2b += Dmb * ut[d];
    wsb += Dmb * (du[d] - dV * n[d]);
    w5b += Dmb * (ut[d] + ct * n[d]);
    utb[d] += Dmb * (w1 + w2 + w5);
    ctb += Dmb * (w5 - w1) * n[d];
    nb[d] += Dmb * ((w5 - w1) * ct - ws * dV);
    dub[d] += Dmb * ws;
    dVb -= Dmb * ws * n[d];
  }
  // Be, De
  rLb += Ge * HL * vnL;
  HLb += Ge * rL * vnL;
  vnLb += Ge * rL * HL;
  rRb += Ge * HR * vnR;
  HRb += Ge * rR * vnR;
  vnRb += Ge * rR * HR;
  {
    const double Deb = -Ge;
    w1b += Deb * (Ht - ct * Vt);
    w2b += Deb * 0.5 * q2t;
    wsb += Deb * (udu - Vt * dV);
    w5b += Deb * (Ht + ct * Vt);
    Htb += Deb * (w1 + w5);
    ctb += Deb * (w5 - w1) * Vt;
    Vtb += Deb * ((w5 - w1) * ct - ws * dV);
    q2tb += Deb * 0.5 * w2;
    udub += Deb * ws;
    dVb -= Deb * ws * Vt;
  }
  const double Ab = 0.5 * hAb;
  // w = m a
  const double m1b = w1b * a1, m5b = w5b * a5, m2b = w2b * a2 + wsb * rt;
  const double a1b = w1b * m1, a5b = w5b * m5, a2b = w2b * m2;
  double rtb = wsb * m2;
  // eigenvalue magnitudes
  double l1b = 0.0, l2b = 0.0, l5b = 0.0;
  if (efix > 0.0) {
    habs_vjp(l1, delta, inv2d, efix, m1b, l1b, ctb);
    habs_vjp(l2, delta, inv2d, efix, m2b, l2b, ctb);
    habs_vjp(l5, delta, inv2d, efix, m5b, l5b, ctb);
  } else {
    l1b = m1b * (l1 > 0.0 ? 1.0 : (l1 < 0.0 ? -1.0 : 0.0));
    l2b = m2b * (l2 > 0.0 ? 1.0 : (l2 < 0.0 ? -1.0 : 0.0));
    l5b = m5b * (l5 > 0.0 ? 1.0 : (l5 < 0.0 ? -1.0 : 0.0));
  }
  Vtb += l1b + l2b + l5b;
  ctb += l5b - l1b;
  // wave strengths
  double dpb = 0.5 * (a1b + a5b) * ic2 - a2b * ic2;
  const double rcdVb = 0.5 * (a5b - a1b) * ic2;
  const double ic2b = 0.5 * a1b * (dp - rcdV) + 0.5 * a5b * (dp + rcdV) - a2b * dp;
  const double drhob = a2b;
  rtb += rcdVb * ct * dV;
  ctb += rcdVb * rt * dV;
  dVb += rcdVb * rt * ct;
  // dV, udu, du
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    dub[d] += dVb * n[d] + udub * ut[d];
    nb[d] += dVb * du[d];
    utb[d] += udub * du[d];
    uRb[d] += dub[d];
    uLb[d] -= dub[d];
  }
  pRb += dpb;
  pLb -= dpb;
  rRb += drhob;
  rLb -= drhob;
  // c~ = sqrt(c2t), 1/c~^2
  const double c2tb = ctb * 0.5 * ict - ic2b * ic2 * ic2;
  Htb += c2tb * g.gm1;
  q2tb -= 0.5 * g.gm1 * c2tb;
  // Vt, q2t, ut
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    utb[d] += Vtb * n[d] + 2.0 * q2tb * ut[d];
    nb[d] += Vtb * ut[d];
  }
  double Rb = 0.0, iR1b = 0.0;
  HLb += Htb * iR1;
  HRb += Htb * R * iR1;
  Rb += Htb * HR * iR1;
  iR1b += Htb * (HL + R * HR);
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    uLb[d] += utb[d] * iR1;
    uRb[d] += utb[d] * R * iR1;
    Rb += utb[d] * uR[d] * iR1;
    iR1b += utb[d] * (uL[d] + R * uR[d]);
  }
  Rb += rtb * rL;
  rLb += rtb * R;
  Rb -= iR1b * iR1 * iR1;
  const double ratiob = Rb * 0.5 * rsq(ratio);  // dR/dratio = 1/(2 sqrt(ratio))
  rRb += ratiob * irL;
  double irLb = ratiob * rR, irRb = 0.0;
  // H = g p / rho + ke / 2
  pLb += HLb * g.g_gm1 * irL;
  irLb += HLb * g.g_gm1 * pL;
  pRb += HRb * g.g_gm1 * irR;
  irRb += HRb * g.g_gm1 * pR;
  rLb -= irLb * irL * irL;
  rRb -= irRb * irR * irR;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    uLb[d] += HLb * uL[d] + vnLb * n[d];  // d(ke/2)/du = u
    uRb[d] += HRb * uR[d] + vnRb * n[d];
    nb[d] += vnLb * uL[d] + vnRb * uR[d];
  }
  // n = S/|S|, A = |S|
  double ndn = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) ndn += nb[d] * n[d];
#pragma unroll
  for (int d = 0; d < DIM; ++d) Sb[d] += Ab * n[d] + (nb[d] - n[d] * ndn) * iA;

  qLb[0] += rLb;
  qRb[0] += rRb;
  qLb[NV - 1] += pLb;
  qRb[NV - 1] += pRb;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    qLb[1 + d] += uLb[d];
    qRb[1 + d] += uRb[d];
  }
}

// Cotangent of the conservative state from the cotangent of the primitive
// state: Qb = (dq/dQ)^T qb at primitive q.
template <int DIM>
__device__ __forceinline__ void prim_cotangent_to_cons(const double* q, const double* qb, const Gas& g, double* Qb) {
  constexpr int NV = DIM + 2;
  const double ir = rcp(q[0]);
  double ke = 0.0, uqb = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    ke += q[1 + d] * q[1 + d];
    uqb += q[1 + d] * qb[1 + d];
  }
  const double pb = qb[NV - 1];
  Qb[0] = qb[0] - uqb * ir + pb * g.gm1 * 0.5 * ke;
#pragma unroll
  for (int d = 0; d < DIM; ++d) Qb[1 + d] = qb[1 + d] * ir - pb * g.gm1 * q[1 + d];
  Qb[NV - 1] = pb * g.gm1;
}

}  // namespace cfd
