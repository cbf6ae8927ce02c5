// Per-face and per-cell arithmetic of the Euler hot path (device functions).
//
// Primitive variables q = (rho, u, v[, w], p); conservative Q = (rho, rho u,
// rho v[, rho w], rho E) with rho E = p/(gamma-1) + rho |u|^2 / 2 (Sec. 2, eq. (2)).
#pragma once

#include <hip/hip_runtime.h>

namespace cfd {

struct Gas {
  double gamma, gm1, igm1, g_gm1;  // gamma, gamma-1, 1/(gamma-1), gamma/(gamma-1)
  double ig, ig2m1;                // 1/gamma, 1/(gamma^2-1)
};

// Reciprocal and reciprocal square root from the hardware estimates (about
// 24 correct bits) refined by one Newton step each, in place of the IEEE
// division / square-root sequences.  Measured on gfx950 over 2^20 arguments
// spread across 20 decades: relative error at most 2.1e-15 (rcp) and 4.1e-15
// (rsq), i.e. a few tens of units in the last place; not correctly rounded.
// Arguments are positive normal numbers on every call site.
__device__ __forceinline__ double rcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Two Newton steps (about one unit in the last place), for the conservative ->
// primitive conversion of every stage, whose round trip rho u / rho must not
// drift over thousands of stages in uniform flow.
__device__ __forceinline__ double rcp2(double x) {
  const double r = rcp(x);
  const double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ double rsq(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-(x * y), y, 1.0);
  return fma(0.5 * y, e, y);
}

// Two Newton steps: the flux-vector splittings scale fluxes by |S| and n, so a
// uniform state's face fluxes sum to zero over a cell only to the accuracy of
// |S| n = S.
__device__ __forceinline__ double rsq2(double x) {
  const double y = rsq(x);
  const double e = fma(-(x * y), y, 1.0);
  return fma(0.5 * y, e, y);
}

// Limiter in slope form S(a, b) = Psi(a / b) * b (defined at b = 0), for the
// symmetric limiters the face states reduce to q_i +- (eps/2) S(D+, D-) for
// every kappa of eq. (flux).  A denominator below 1e-250 returns 0: the
// differences are then below 1e-250 (van Leer) or 1e-125 (van Albada without
// regularisation) and so is the exact slope.
// LIM_VANALBADA0: van Albada with every regularisation e = 0, a stage-kernel
// specialisation with the e^2 terms compiled out (the same bits: fma(a, a, 0)
// is the rounded product), which frees the registers the e^2 values held.
enum { LIM_NONE = 0, LIM_VANLEER = 1, LIM_VANALBADA = 2, LIM_FROZEN = 3, LIM_VANALBADA0 = 4 };
constexpr double SLOPE_TINY = 1e-250;

template <int LIM>
__device__ __forceinline__ double slope(double a, double b, double e2) {
  if constexpr (LIM == LIM_NONE) {
    return b;
  } else if constexpr (LIM == LIM_VANLEER) {
    double aa = fabs(a), ab = fabs(b);
    double den = aa + ab;
    double num = a * ab + aa * b;
    return den > SLOPE_TINY ? num * rcp(den) : 0.0;
  } else {
    // with A = a^2 + e^2, B = b^2 + e^2: S = (B a + A b) / (A + B)
    const double A = LIM == LIM_VANALBADA0 ? a * a : fma(a, a, e2);
    const double B = LIM == LIM_VANALBADA0 ? b * b : fma(b, b, e2);
    const double den = A + B;
    const double num = fma(B, a, A * b);
    return den > SLOPE_TINY ? num * rcp(den) : 0.0;
  }
}

// Per-cell slopes of eq. (flux) for the two faces of a cell along one
// direction, from the backward and forward differences dm = q_i - q_{i-1},
// dp = q_{i+1} - q_i:  q^L_{i+1/2} = q_i + (eps/2) sp,  q^R_{i-1/2} = q_i - (eps/2) sm.
// Symmetric limiters: sp = sm = S(dp, dm) for every kappa.  Psi = 1 (no limiter):
// sp = ((1-kappa) dm + (1+kappa) dp)/2, sm = ((1+kappa) dm + (1-kappa) dp)/2.
template <int LIM>
__device__ __forceinline__ void cell_slopes(double dm, double dp, double e2, double kap, double& sp, double& sm) {
  if constexpr (LIM == LIM_NONE) {
    sp = 0.5 * ((1.0 - kap) * dm + (1.0 + kap) * dp);
    sm = 0.5 * ((1.0 + kap) * dm + (1.0 - kap) * dp);
  } else {
    sp = slope<LIM>(dp, dm, e2);
    sm = sp;
  }
}

// Limiter freezing: the frozen factor phi = S(a, b) / ((a + b)/2) of a cell
// (a, b its forward and backward differences at the freeze), in closed form:
// van Leer 4ab/(a + b)^2 for ab > 0, else 0; van Albada
// 2(ab + e^2)/(a^2 + b^2 + 2e^2), 0 where a + b = 0 (S vanishes there).
// Frozen, the slope is phi (a + b)/2 with the current differences.
template <int LIM>
__device__ __forceinline__ double frozen_factor(double a, double b, double e2) {
  if constexpr (LIM == LIM_VANLEER) {
    const double ab = a * b, s = a + b;
    return ab > 0.0 ? 4.0 * ab / (s * s) : 0.0;
  } else {
    if (a + b == 0.0) return 0.0;
    return 2.0 * (a * b + e2) / (a * a + b * b + 2.0 * e2);
  }
}
__device__ __forceinline__ double frozen_slope(double phi, double dm, double dp) { return phi * (0.5 * (dm + dp)); }

template <int DIM>
__device__ __forceinline__ void prim_to_cons(const double* q, const Gas& g, double* Q) {
  double ke = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) ke += q[1 + d] * q[1 + d];
  Q[0] = q[0];
#pragma unroll
  for (int d = 0; d < DIM; ++d) Q[1 + d] = q[0] * q[1 + d];
  Q[DIM + 1] = q[DIM + 1] * g.igm1 + 0.5 * q[0] * ke;
}

template <int DIM>
__device__ __forceinline__ void cons_to_prim(const double* Q, const Gas& g, double* q) {
  double ir = rcp2(Q[0]);
  double ke = 0.0;
  q[0] = Q[0];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    q[1 + d] = Q[1 + d] * ir;
    ke += q[1 + d] * q[1 + d];
  }
  q[DIM + 1] = g.gm1 * (Q[DIM + 1] - 0.5 * Q[0] * ke);
}

// Harten-smoothed absolute value: |l| where |l| >= delta, else (l^2 + delta^2) / (2 delta).
__device__ __forceinline__ double habs(double l, double delta, double inv2d) {
  double a = fabs(l);
  return a >= delta ? a : (l * l + delta * delta) * inv2d;
}

// Roe flux-difference splitting (Sec. 2; textbook rotated form) through a
// face with area vector S (|S| = area, S/|S| = unit normal toward the right
// state).  Output: flux times area.  efix > 0 enables Harten smoothing of all
// three eigenvalue families with half-width efix * c~.
template <int DIM>
__device__ __forceinline__ void roe_flux(const double* qL, const double* qR, const double* S, const Gas& g,
                                         double efix, double half_inv_efix, double* F) {
  constexpr int NV = DIM + 2;
  double A2 = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) A2 += S[d] * S[d];
  const double iA = rsq(A2);  // 1/|S|
  const double A = A2 * iA;
  double n[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) n[d] = S[d] * iA;

  const double rL = qL[0], rR = qR[0];
  const double pL = qL[NV - 1], pR = qR[NV - 1];
  // normal velocities times area (u . S): the central flux is formed from S
  // directly, so a uniform state gives exactly the central flux whatever the
  // rounding of |S| and n (freestream preservation rests on the metrics alone)
  double vsL = 0.0, vsR = 0.0, keL = 0.0, keR = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    vsL += qL[1 + d] * S[d];
    vsR += qR[1 + d] * S[d];
    keL += qL[1 + d] * qL[1 + d];
    keR += qR[1 + d] * qR[1 + d];
  }
  const double irL = rcp(rL), irR = rcp(rR);
  const double HL = g.g_gm1 * pL * irL + 0.5 * keL;
  const double HR = g.g_gm1 * pR * irR + 0.5 * keR;

  // Roe averages, R = sqrt(rho_R / rho_L)
  const double ratio = rR * irL;
  const double R = ratio * rsq(ratio);
  const double iR1 = rcp(1.0 + R);
  const double rt = R * rL;
  double ut[DIM];
  double q2t = 0.0, Vt = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    ut[d] = (qL[1 + d] + R * qR[1 + d]) * iR1;
    q2t += ut[d] * ut[d];
    Vt += ut[d] * n[d];
  }
  const double Ht = (HL + R * HR) * iR1;
  const double c2t = g.gm1 * (Ht - 0.5 * q2t);
  const double ict = rsq(c2t);  // 1/c~
  const double ct = c2t * ict;
  const double ic2 = ict * ict;

  // jumps and wave strengths
  const double drho = rR - rL;
  const double dp = pR - pL;
  double du[DIM];
  double dV = 0.0, udu = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    du[d] = qR[1 + d] - qL[1 + d];
    dV += du[d] * n[d];
    udu += ut[d] * du[d];
  }
  const double rcdV = rt * ct * dV;
  const double a1 = 0.5 * (dp - rcdV) * ic2;
  const double a5 = 0.5 * (dp + rcdV) * ic2;
  const double a2 = drho - dp * ic2;

  double m1, m2, m5;
  if (efix > 0.0) {
    const double delta = efix * ct;
    const double inv2d = half_inv_efix * ict;  // 1 / (2 delta)
    m1 = habs(Vt - ct, delta, inv2d);
    m2 = habs(Vt, delta, inv2d);
    m5 = habs(Vt + ct, delta, inv2d);
  } else {
    m1 = fabs(Vt - ct);
    m2 = fabs(Vt);
    m5 = fabs(Vt + ct);
  }
  const double w1 = m1 * a1, w5 = m5 * a5, w2 = m2 * a2, ws = m2 * rt;

  // dissipation sum_k w_k r_k with the eigenvectors r_1,5 = (1, u~ -+ c~ n,
  // H~ -+ c~ V~), r_2 = (1, u~, q~^2/2) and the shear part ws (du - dV n,
  // u~.du - V~ dV), collected by term: W = w1 + w2 + w5 multiplies u~,
  // Wc = (w5 - w1) c~ multiplies n and V~; central part per component
  const double W = w1 + w2 + w5;
  const double Wc = (w5 - w1) * ct;
  const double Wn = Wc - ws * dV;
  const double mL = rL * vsL, mR = rR * vsR, P = pL + pR;  // mass fluxes times area
  const double hA = 0.5 * A;
  F[0] = 0.5 * (mL + mR) - hA * W;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const double Dm = W * ut[d] + Wn * n[d] + ws * du[d];
    F[1 + d] = 0.5 * (mL * qL[1 + d] + mR * qR[1 + d] + P * S[d]) - hA * Dm;
  }
  const double De = (W - w2) * Ht + Wc * Vt + w2 * 0.5 * q2t + ws * (udu - Vt * dV);
  F[NV - 1] = 0.5 * (mL * HL + mR * HR) - hA * De;
}

// ---------------------------------------------------------------------------
// Flux-vector splittings (Sec. 2 lists van Leer's and Steger and Warming's;
// textbook forms).  Face flux A (F+(qL) + F-(qR)) with A = |S|, n = S / A.

enum { FLUX_ROE = 0, FLUX_VANLEER_FVS = 1, FLUX_STEGER_WARMING = 2 };

// Steger-Warming part F+ (sign = 1) or F- (sign = -1) per unit area, added to F:
// F+- = rho/(2 gamma) [a, a u + c (l3 - l1) n, a |u|^2/2 + c V (l3 - l1) + c^2 (l1 + l3)/(gamma-1)],
// a = 2 (gamma-1) l2 + l1 + l3, each eigenvalue l1,2,3 = V - c, V, V + c taken as (l +- |l|)/2.
template <int DIM>
__device__ __forceinline__ void steger_warming_part(const double* q, const double* n, double sign, const Gas& g,
                                                    double* F) {
  constexpr int NV = DIM + 2;
  const double rho = q[0], p = q[NV - 1];
  const double c2 = g.gamma * p * rcp(rho);
  const double c = c2 * rsq(c2);
  double V = 0.0, q2 = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    V += q[1 + d] * n[d];
    q2 += q[1 + d] * q[1 + d];
  }
  const double l1 = 0.5 * ((V - c) + sign * fabs(V - c));
  const double l2 = 0.5 * (V + sign * fabs(V));
  const double l3 = 0.5 * ((V + c) + sign * fabs(V + c));
  const double a = 2.0 * g.gm1 * l2 + l1 + l3;
  const double k = 0.5 * rho * g.ig;
  const double d31 = c * (l3 - l1);
  F[0] += k * a;
#pragma unroll
  for (int d = 0; d < DIM; ++d) F[1 + d] += k * (a * q[1 + d] + d31 * n[d]);
  F[NV - 1] += k * (a * 0.5 * q2 + d31 * V + c2 * (l1 + l3) * g.igm1);
}

// van Leer part per unit area, added to F: the full flux beyond Mach 1 on its
// own side, nothing beyond Mach 1 on the other, else with M = V/c and the mass
// flux f = +-rho c (M +- 1)^2 / 4:
// F+- = f [1, u + n (-V +- 2c)/gamma, (|u|^2 - V^2)/2 + ((gamma-1) V +- 2c)^2 / (2 (gamma^2 - 1))].
template <int DIM>
__device__ __forceinline__ void van_leer_part(const double* q, const double* n, double sign, const Gas& g,
                                              double* F) {
  constexpr int NV = DIM + 2;
  const double rho = q[0], p = q[NV - 1];
  const double irho = rcp(rho);
  const double c2 = g.gamma * p * irho;
  const double ic = rsq(c2);
  const double c = c2 * ic;
  double V = 0.0, q2 = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    V += q[1 + d] * n[d];
    q2 += q[1 + d] * q[1 + d];
  }
  const double M = V * ic;
  const double sM = sign * M;
  if (sM >= 1.0) {  // supersonic towards this side: the whole flux
    F[0] += rho * V;
#pragma unroll
    for (int d = 0; d < DIM; ++d) F[1 + d] += rho * q[1 + d] * V + p * n[d];
    F[NV - 1] += (g.g_gm1 * p + 0.5 * rho * q2) * V;
  } else if (sM > -1.0) {
    const double mp = M + sign;
    const double f = sign * 0.25 * rho * c * mp * mp;
    const double vn = (-V + sign * 2.0 * c) * g.ig;
    const double t = g.gm1 * V + sign * 2.0 * c;
    F[0] += f;
#pragma unroll
    for (int d = 0; d < DIM; ++d) F[1 + d] += f * (q[1 + d] + vn * n[d]);
    F[NV - 1] += f * (0.5 * (q2 - V * V) + 0.5 * t * t * g.ig2m1);
  }
}

template <int DIM, int FLUX>
__device__ __forceinline__ void fvs_flux(const double* qL, const double* qR, const double* S, const Gas& g,
                                         double* F) {
  constexpr int NV = DIM + 2;
  double A2 = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) A2 += S[d] * S[d];
  const double iA = rsq2(A2);
  const double A = A2 * iA;
  double n[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) n[d] = S[d] * iA;
  double G[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) G[v] = 0.0;
  if constexpr (FLUX == FLUX_VANLEER_FVS) {
    van_leer_part<DIM>(qL, n, 1.0, g, G);
    van_leer_part<DIM>(qR, n, -1.0, g, G);
  } else {
    steger_warming_part<DIM>(qL, n, 1.0, g, G);
    steger_warming_part<DIM>(qR, n, -1.0, g, G);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) F[v] = A * G[v];
}

// face flux of the configured scheme
template <int DIM, int FLUX>
__device__ __forceinline__ void face_flux(const double* qL, const double* qR, const double* S, const Gas& g,
                                          double efix, double half_inv_efix, double* F) {
  if constexpr (FLUX == FLUX_ROE)
    roe_flux<DIM>(qL, qR, S, g, efix, half_inv_efix, F);
  else
    fvs_flux<DIM, FLUX>(qL, qR, S, g, F);
}

}  // namespace cfd
