// Residual vector-Jacobian product (adjoint) kernels.
//
// R(Q) = ghost fill -> MUSCL face states -> Roe / wall flux -> divergence
// (the forward path of stage_kernel.h).  Given Rb = dJ/dR the passes below
// return dJ/dQ, accumulate dJ/dS (face area vectors) and dJ/dOmega (cell
// volumes) for the node gradient, and dJ/dtheta for inflow states.  Every pass
// is a gather with a unique writer per output element, so results do not
// depend on scheduling:
//   1. face pass: per face, the flux VJP -> cotangents of the two
//      reconstructed face states (or of the wall pressure), dJ/dS, and the two
//      scalars sum_v Rb_v F_v that feed dJ/d(1/Omega);
//   2. cell pass: per padded cell, gathers the face-state cotangents through
//      the limited slopes of its own and its two neighbours' stencils;
//   3. ghost transposes, one launch per donor face so no two threads add into
//      the same cell: connections copy ghost cotangents back to their donor
//      cells, mirror walls reflect them (and add the wall-normal term to
//      dJ/dS), outflow copies add to the adjacent cell, inflow ghosts sum into
//      per-patch partials;
//   4. finalize: primitive -> conservative cotangent per interior cell.
#include <hip/hip_runtime.h>

#include "adjoint.h"
#include "adjoint_math.h"
#include "cfd_internal.h"

namespace cfd {

__device__ __forceinline__ long long axis_step(const BlockDev& B, int d) {
  return d == 0 ? 1LL : (d == 1 ? (long long)B.pi : (long long)B.pi * B.pj);
}

__device__ __forceinline__ int ext(const BlockDev& B, int d) { return d == 0 ? B.ni : (d == 1 ? B.nj : B.nk); }

__device__ __forceinline__ bool wall_at(const VjpArgs& a, int b, int face, int t1, int t2) {
  for (int p = 0; p < a.npatches; ++p) {
    const PatchDev& pt = a.patches[p];
    if (pt.block == b && pt.face == face && pt.kind == PK_SLIP_WALL && t1 >= pt.lo0 && t1 < pt.lo0 + pt.len0 &&
        t2 >= pt.lo1 && t2 < pt.lo1 + pt.len1)
      return true;
  }
  return false;
}

// tangential coordinates of cell (i,j,k) with respect to an axis-d face
__device__ __forceinline__ void tang(int d, int i, int j, int k, int& t1, int& t2) {
  t1 = d == 0 ? j : i;
  t2 = d == 2 ? j : k;
}

// ---------------------------------------------------------------------------
// 1. face pass

template <int DIM, int LIM>
__global__ void __launch_bounds__(256) vjp_face_kernel(VjpArgs a) {
  constexpr int NV = DIM + 2;
  using ML = MetricLayout<DIM>;
  const int b = blockIdx.y;
  const BlockDev B = a.blocks[b];
  long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  // faces of direction 0, then 1, then 2
  int d = -1;
  int e0 = 1, e1 = 1, e2 = 1;
  for (int dd = 0; dd < DIM; ++dd) {
    const int x0 = B.ni + (dd == 0), x1 = B.nj + (dd == 1), x2 = DIM == 3 ? B.nk + (dd == 2) : 1;
    const long long nf = (long long)x0 * x1 * x2;
    if (c < nf) {
      d = dd;
      e0 = x0;
      e1 = x1;
      e2 = x2;
      break;
    }
    c -= nf;
  }
  if (d < 0) return;
  const int i = (int)(c % e0), j = (int)((c / e0) % e1), k = (int)(c / ((long long)e0 * e1));
  (void)e2;
  const long long st = axis_step(B, d);
  const int f = d == 0 ? i : (d == 1 ? j : k);  // face index along d; cells L = f-1, R = f
  const int n = ext(B, d);
  const long long fidx = pidx(B, i, j, k);  // face position == cell R position
  const long long vs = B.vstride;
  const double* q = a.q + B.origin + fidx;
  const double* met = a.metric + B.morigin + fidx;
  double qm[NV], qa[NV], qb[NV], qp[NV];  // cells L-1, L, R, R+1
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    qm[v] = q[v * vs - 2 * st];
    qa[v] = q[v * vs - st];
    qb[v] = q[v * vs];
    qp[v] = q[v * vs + st];
  }
  double S[DIM];
#pragma unroll
  for (int cc = 0; cc < DIM; ++cc) S[cc] = met[ML::S(d, cc) * vs];
  // flux cotangent Fb = Rb_L * invvol_L - Rb_R * invvol_R (interior cells only)
  const bool Lin = f >= 1, Rin = f < n;
  double Fb[NV], RbL[NV], RbR[NV];
  const long long pcR = B.packed + ((long long)k * B.nj + j) * B.ni + i;
  const long long pcL = pcR - (d == 0 ? 1LL : (d == 1 ? (long long)B.ni : (long long)B.ni * B.nj));
  const double ivL = Lin ? met[ML::INVVOL * vs - st] : 0.0;
  const double ivR = Rin ? met[ML::INVVOL * vs] : 0.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    RbL[v] = Lin ? a.Rb[v * B.ncell_total + pcL] : 0.0;
    RbR[v] = Rin ? a.Rb[v * B.ncell_total + pcR] : 0.0;
    Fb[v] = RbL[v] * ivL - RbR[v] * ivR;
  }
  int t1, t2;
  tang(d, i, j, k, t1, t2);
  const int face = f == 0 ? 2 * d : (f == n ? 2 * d + 1 : -1);
  double F[NV], Lb[NV], Rb_[NV], Sb[DIM];
#pragma unroll
  for (int v = 0; v < NV; ++v) Lb[v] = Rb_[v] = 0.0;
#pragma unroll
  for (int cc = 0; cc < DIM; ++cc) Sb[cc] = 0.0;
  double pwb = 0.0;
  double* fb = a.facebar + B.forigin + fidx;
  const int base = d * (2 * NV + 3);
  if (face >= 0 && (B.wall_mask & (1 << face)) && wall_at(a, b, face, t1, t2)) {
    // F = (0, p_w S, 0), p_w = 1.5 p0 - 0.5 p1 with p0 the cell next to the wall
    const double p0 = (face & 1) ? qa[NV - 1] : qb[NV - 1];
    const double p1 = (face & 1) ? qm[NV - 1] : qp[NV - 1];
    const double pw = 1.5 * p0 - 0.5 * p1;
    F[0] = F[NV - 1] = 0.0;
#pragma unroll
    for (int cc = 0; cc < DIM; ++cc) {
      F[1 + cc] = pw * S[cc];
      pwb += Fb[1 + cc] * S[cc];
      Sb[cc] += pw * Fb[1 + cc];
    }
  } else {
    double qL[NV], qR[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double spa, sma, spb, smb;
      cell_slopes<LIM>(qa[v] - qm[v], qb[v] - qa[v], a.e2[v], a.kappa, spa, sma);
      cell_slopes<LIM>(qb[v] - qa[v], qp[v] - qb[v], a.e2[v], a.kappa, spb, smb);
      qL[v] = qa[v] + a.half_eps * spa;
      qR[v] = qb[v] - a.half_eps * smb;
    }
    roe_flux_vjp<DIM>(qL, qR, S, a.gas, a.efix, a.half_inv_efix, Fb, F, Lb, Rb_, Sb);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    fb[(base + v) * vs] = Lb[v];
    fb[(base + NV + v) * vs] = Rb_[v];
  }
  fb[(base + 2 * NV) * vs] = pwb;
  double cL = 0.0, cR = 0.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    cL += RbL[v] * F[v];
    cR -= RbR[v] * F[v];
  }
  fb[(base + 2 * NV + 1) * vs] = cL;
  fb[(base + 2 * NV + 2) * vs] = cR;
  double* mb = a.metricbar + B.morigin + fidx;
#pragma unroll
  for (int cc = 0; cc < DIM; ++cc) mb[ML::S(d, cc) * vs] += a.scale * Sb[cc];
}

// ---------------------------------------------------------------------------
// 2. cell pass

template <int DIM, int LIM>
__global__ void __launch_bounds__(256) vjp_cell_kernel(VjpArgs a) {
  constexpr int NV = DIM + 2;
  using ML = MetricLayout<DIM>;
  const int b = blockIdx.y;
  const BlockDev B = a.blocks[b];
  const int ei = B.ni + 4, ej = B.nj + 4, ek = DIM == 3 ? B.nk + 4 : 1;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long long)ei * ej * ek) return;
  const int i = (int)(c % ei) - 2, j = (int)((c / ei) % ej) - 2;
  const int k = DIM == 3 ? (int)(c / ((long long)ei * ej)) - 2 : 0;
  const int co[3] = {i, j, k};
  const int nn[3] = {B.ni, B.nj, B.nk};
  int nout = 0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) nout += (co[d] < 0 || co[d] >= nn[d]);
  if (nout > 1) return;  // corner ghosts take no part
  const long long ci = pidx(B, i, j, k);
  const long long vs = B.vstride;
  const double* q = a.q + B.origin + ci;
  const double* fb = a.facebar + B.forigin + ci;
  double qb[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) qb[v] = 0.0;
  double ivb = 0.0;
  for (int d = 0; d < DIM; ++d) {
    bool others_in = true;
#pragma unroll
    for (int e = 0; e < DIM; ++e)
      if (e != d) others_in = others_in && co[e] >= 0 && co[e] < nn[e];
    if (!others_in) continue;
    const int n = nn[d];
    const int x = co[d];
    const long long st = axis_step(B, d);
    const int base = d * (2 * NV + 3);
    // face m lies between cells m-1 and m; valid for 0 <= m <= n
    auto Lbar = [&](int m, int v) -> double {  // cotangent of q^L at face m
      return (m >= 0 && m <= n) ? fb[(base + v) * vs + (long long)(m - x) * st] : 0.0;
    };
    auto Rbar = [&](int m, int v) -> double {  // cotangent of q^R at face m
      return (m >= 0 && m <= n) ? fb[(base + NV + v) * vs + (long long)(m - x) * st] : 0.0;
    };
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      // direct dependence: cell x is the left state of face x+1 and the right state of face x
      qb[v] += Lbar(x + 1, v) + Rbar(x, v);
      // slopes of cells m = x-1, x, x+1 depend on q_x
      for (int m = x - 1; m <= x + 1; ++m) {
        const bool hp = (m + 1 >= 0 && m + 1 <= n);  // sigma+_m used at face m+1
        const bool hm = (m >= 0 && m <= n);          // sigma-_m used at face m
        if (!hp && !hm) continue;
        const double spb = hp ? a.half_eps * Lbar(m + 1, v) : 0.0;
        const double smb = hm ? -a.half_eps * Rbar(m, v) : 0.0;
        if (spb == 0.0 && smb == 0.0) continue;
        const double qm1 = q[v * vs + (long long)(m - 1 - x) * st];
        const double q0 = q[v * vs + (long long)(m - x) * st];
        const double qp1 = q[v * vs + (long long)(m + 1 - x) * st];
        double gp, hmv;
        slope_vjp<LIM>(q0 - qm1, qp1 - q0, a.e2[v], a.kappa, spb, smb, gp, hmv);
        // dp_m = q_{m+1} - q_m, dm_m = q_m - q_{m-1}
        if (m == x - 1) qb[v] += gp;
        if (m == x) qb[v] += hmv - gp;
        if (m == x + 1) qb[v] -= hmv;
      }
    }
    if (x >= 0 && x < n) {
      // wall pressure extrapolation p_w = 1.5 p0 - 0.5 p1 on wall faces 0 and n
      int t1, t2;
      tang(d, i, j, k, t1, t2);
      if ((x == 0 || x == 1) && (B.wall_mask & (1 << (2 * d))) && wall_at(a, b, 2 * d, t1, t2))
        qb[NV - 1] += (x == 0 ? 1.5 : -0.5) * fb[(base + 2 * NV) * vs + (long long)(0 - x) * st];
      if ((x == n - 1 || x == n - 2) && (B.wall_mask & (1 << (2 * d + 1))) && wall_at(a, b, 2 * d + 1, t1, t2))
        qb[NV - 1] += (x == n - 1 ? 1.5 : -0.5) * fb[(base + 2 * NV) * vs + (long long)(n - x) * st];
      // 1/Omega: the cell is the left cell of face x+1 and the right cell of face x
      ivb += fb[(base + 2 * NV + 1) * vs + st] + fb[(base + 2 * NV + 2) * vs];
    }
  }
  double* out = a.qbar + B.origin + ci;
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v * vs] = qb[v];
  bool interior = true;
#pragma unroll
  for (int d = 0; d < DIM; ++d) interior = interior && co[d] >= 0 && co[d] < nn[d];
  if (interior) {
    // Omega-bar = -(1/Omega)-bar / Omega^2
    const double iv = a.metric[B.morigin + ML::INVVOL * vs + ci];
    a.metricbar[B.morigin + ML::INVVOL * vs + ci] += a.scale * (-ivb * iv * iv);
  }
}

// ---------------------------------------------------------------------------
// 3. ghost transposes (launch per donor face)

template <int DIM>
__global__ void __launch_bounds__(CHUNK) vjp_ghost_kernel(VjpArgs a, const ChunkDev* chunks, int chunk_begin) {
  constexpr int NV = DIM + 2;
  using ML = MetricLayout<DIM>;
  const ChunkDev ch = chunks[chunk_begin + blockIdx.x];
  if ((int)threadIdx.x >= ch.count) return;
  const int e = ch.start + threadIdx.x;  // tangential position index
  if (ch.kind == 0) {
    const TransferDev x = a.xfers[ch.item];
    const int r1 = e % x.len0, r2 = e / x.len0;
    int d1, d2;
    orient_map(x.orient, r1, r2, x.dlen0, x.dlen1, d1, d2);
    const BlockDev& D = a.blocks[x.dblock];
    const BlockDev& R = a.blocks[x.rblock];
    for (int g = 0; g < NG; ++g) {
      int di, dj, dk, gi, gj, gk;
      face_cell(D, DIM, x.dface, g, false, x.dlo0 + d1, x.dlo1 + d2, di, dj, dk);
      face_cell(R, DIM, x.rface, g, true, x.rlo0 + r1, x.rlo1 + r2, gi, gj, gk);
      double* dst = a.qbar + D.origin + pidx(D, di, dj, dk);
      const double* src = a.qbar + R.origin + pidx(R, gi, gj, gk);
#pragma unroll
      for (int v = 0; v < NV; ++v) dst[v * D.vstride] += src[v * R.vstride];
    }
    return;
  }
  const PatchDev p = a.patches[ch.item];
  const int t1 = p.lo0 + e % p.len0, t2 = p.lo1 + e / p.len0;
  const BlockDev& B = a.blocks[p.block];
  const long long vs = B.vstride;
  double* qb = a.qbar + B.origin;
  if (p.kind == PK_SUP_INFLOW) {
    double s[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] = 0.0;
    for (int g = 0; g < NG; ++g) {
      int gi, gj, gk;
      face_cell(B, DIM, p.face, g, true, t1, t2, gi, gj, gk);
      const long long gidx = pidx(B, gi, gj, gk);
#pragma unroll
      for (int v = 0; v < NV; ++v) s[v] += qb[v * vs + gidx];
    }
    double* part = a.inflow_part + a.part_offset[ch.item];
#pragma unroll
    for (int v = 0; v < NV; ++v) part[v * p.len0 * p.len1 + e] = s[v];
    return;
  }
  if (p.kind == PK_EXTRAP_OUTFLOW) {
    int si, sj, sk;
    face_cell(B, DIM, p.face, 0, false, t1, t2, si, sj, sk);
    const long long sidx = pidx(B, si, sj, sk);
    for (int g = 0; g < NG; ++g) {
      int gi, gj, gk;
      face_cell(B, DIM, p.face, g, true, t1, t2, gi, gj, gk);
      const long long gidx = pidx(B, gi, gj, gk);
#pragma unroll
      for (int v = 0; v < NV; ++v) qb[v * vs + sidx] += qb[v * vs + gidx];
    }
    return;
  }
  // slip wall: ghost g = mirror of interior g about the wall face
  int fi, fj, fk;
  face_cell(B, DIM, p.face, 0, (p.face & 1) != 0, t1, t2, fi, fj, fk);
  const long long fidx = pidx(B, fi, fj, fk);
  double S[DIM], Sb[DIM];
  double s2 = 0.0;
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    S[c] = a.metric[B.morigin + ML::S(p.face >> 1, c) * vs + fidx];
    s2 += S[c] * S[c];
    Sb[c] = 0.0;
  }
  const double is2 = 1.0 / s2;
  for (int g = 0; g < NG; ++g) {
    int gi, gj, gk, mi, mj, mk;
    face_cell(B, DIM, p.face, g, true, t1, t2, gi, gj, gk);
    face_cell(B, DIM, p.face, g, false, t1, t2, mi, mj, mk);
    const long long gidx = pidx(B, gi, gj, gk), midx = pidx(B, mi, mj, mk);
    double ug[DIM], um[DIM];
    double un = 0.0, ugS = 0.0;
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      ug[c] = qb[(1 + c) * vs + gidx];                       // cotangent of the ghost velocity
      um[c] = a.q[B.origin + (1 + c) * vs + midx];          // interior velocity
      un += um[c] * S[c];
      ugS += ug[c] * S[c];
    }
    // u_g = u_m - f S with f = 2 (u_m . S) / |S|^2
    const double fco = 2.0 * un * is2;
    qb[midx] += qb[gidx];
    qb[(NV - 1) * vs + midx] += qb[(NV - 1) * vs + gidx];
#pragma unroll
    for (int c = 0; c < DIM; ++c) qb[(1 + c) * vs + midx] += ug[c] - 2.0 * ugS * S[c] * is2;
    // dJ/dS: -f ug_k - (ug . S) (2 u_k / |S|^2 - 4 (u . S) S_k / |S|^4)
#pragma unroll
    for (int c = 0; c < DIM; ++c) Sb[c] += -fco * ug[c] - ugS * (2.0 * um[c] * is2 - 4.0 * un * S[c] * is2 * is2);
  }
  double* mb = a.metricbar + B.morigin;
#pragma unroll
  for (int c = 0; c < DIM; ++c) mb[ML::S(p.face >> 1, c) * vs + fidx] += a.scale * Sb[c];
}

// ---------------------------------------------------------------------------
// 4. finalize: Qb = scale * (dq/dQ)^T qb ; out = Qb ; acc += Qb

template <int DIM>
__global__ void vjp_finalize_kernel(VjpArgs a) {
  constexpr int NV = DIM + 2;
  const BlockDev B = a.blocks[blockIdx.y];
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = (long long)B.ni * B.nj * B.nk;
  if (c >= n) return;
  const int i = (int)(c % B.ni);
  const int j = (int)((c / B.ni) % B.nj);
  const int k = (int)(c / ((long long)B.ni * B.nj));
  const long long ci = pidx(B, i, j, k);
  double q[NV], qb[NV], Qb[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    q[v] = a.q[B.origin + v * B.vstride + ci];
    qb[v] = a.qbar[B.origin + v * B.vstride + ci];
  }
  prim_cotangent_to_cons<DIM>(q, qb, a.gas, Qb);
  const long long pc = B.packed + c;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double val = a.scale * Qb[v];
    if (a.out) a.out[v * B.ncell_total + pc] = val;
    if (a.acc) a.acc[v * B.ncell_total + pc] += val;
  }
}

// inflow partial sums -> theta-bar (one workgroup per inflow patch, fixed order)
template <int DIM>
__global__ void __launch_bounds__(256) vjp_inflow_reduce_kernel(VjpArgs a, const int* inflow_patches) {
  constexpr int NV = DIM + 2;
  __shared__ double red[256];
  const int pi_ = inflow_patches[blockIdx.x];
  const PatchDev p = a.patches[pi_];
  const int cnt = p.len0 * p.len1;
  const double* part = a.inflow_part + a.part_offset[pi_];
  for (int v = 0; v < NV; ++v) {
    double s = 0.0;
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) s += part[v * cnt + t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.thetabar[p.param * MAXV + v] += a.scale * red[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// objective: J = sum over slip-wall faces of p_w |S| (launch per wall face f)

template <int DIM>
__global__ void __launch_bounds__(CHUNK) objective_kernel(VjpArgs a, const ChunkDev* chunks, int chunk_begin) {
  constexpr int NV = DIM + 2;
  using ML = MetricLayout<DIM>;
  const ChunkDev ch = chunks[chunk_begin + blockIdx.x];
  if ((int)threadIdx.x >= ch.count) return;
  const int e = ch.start + threadIdx.x;
  const PatchDev p = a.patches[ch.item];
  const int t1 = p.lo0 + e % p.len0, t2 = p.lo1 + e / p.len0;
  const BlockDev& B = a.blocks[p.block];
  const long long vs = B.vstride;
  int i0, j0, k0, i1, j1, k1, fi, fj, fk;
  face_cell(B, DIM, p.face, 0, false, t1, t2, i0, j0, k0);
  face_cell(B, DIM, p.face, 1, false, t1, t2, i1, j1, k1);
  face_cell(B, DIM, p.face, 0, (p.face & 1) != 0, t1, t2, fi, fj, fk);
  const long long c0 = pidx(B, i0, j0, k0), c1 = pidx(B, i1, j1, k1), fidx = pidx(B, fi, fj, fk);
  const double p0 = a.q[B.origin + (NV - 1) * vs + c0];
  const double p1 = a.q[B.origin + (NV - 1) * vs + c1];
  const double pw = 1.5 * p0 - 0.5 * p1;
  double S[DIM], s2 = 0.0;
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    S[c] = a.metric[B.morigin + ML::S(p.face >> 1, c) * vs + fidx];
    s2 += S[c] * S[c];
  }
  const double A = sqrt(s2);
  a.inflow_part[a.part_offset[ch.item] + e] = pw * A;
  a.qbar[B.origin + (NV - 1) * vs + c0] += 1.5 * A;
  a.qbar[B.origin + (NV - 1) * vs + c1] += -0.5 * A;
#pragma unroll
  for (int c = 0; c < DIM; ++c) a.metricbar[B.morigin + ML::S(p.face >> 1, c) * vs + fidx] += pw * S[c] / A;
}

__global__ void __launch_bounds__(256) objective_sum_kernel(VjpArgs a, const int* wall_patches, int nwall, double* J) {
  __shared__ double red[256];
  double s = 0.0;
  for (int w = 0; w < nwall; ++w) {
    const PatchDev p = a.patches[wall_patches[w]];
    const int cnt = p.len0 * p.len1;
    const double* part = a.inflow_part + a.part_offset[wall_patches[w]];
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) s += part[t];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) J[0] = red[0];
}

// ---------------------------------------------------------------------------
// node gradient (2D): gather dJ/dS and dJ/dOmega onto the nodes

__global__ void node_vjp_2d_kernel(VjpArgs a, double* Xb) {
  using ML = MetricLayout<2>;
  const BlockDev B = a.blocks[blockIdx.y];
  const int ni1 = B.ni + 1, nj1 = B.nj + 1;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long long)ni1 * nj1) return;
  const int i = (int)(c % ni1), j = (int)(c / ni1);
  const long long vs = B.vstride;
  const double* mb = a.metricbar + B.morigin;
  const long long nn = B.nnode_total;
  auto X = [&](int cc, int ii, int jj) -> double { return a.nodes[cc * nn + B.node0 + (long long)jj * ni1 + ii]; };
  double xb = 0.0, yb = 0.0;
  // i-face (i, j): nodes (i,j) -> (i,j+1), S = (y1 - y0, -(x1 - x0))
  if (j < B.nj) {
    const long long f = pidx(B, i, j, 0);
    xb += mb[ML::S(0, 1) * vs + f];
    yb -= mb[ML::S(0, 0) * vs + f];
  }
  if (j > 0) {
    const long long f = pidx(B, i, j - 1, 0);
    xb -= mb[ML::S(0, 1) * vs + f];
    yb += mb[ML::S(0, 0) * vs + f];
  }
  // j-face (i, j): nodes (i,j) -> (i+1,j), S = (-(y1 - y0), x1 - x0)
  if (i < B.ni) {
    const long long f = pidx(B, i, j, 0);
    xb -= mb[ML::S(1, 1) * vs + f];
    yb += mb[ML::S(1, 0) * vs + f];
  }
  if (i > 0) {
    const long long f = pidx(B, i - 1, j, 0);
    xb += mb[ML::S(1, 1) * vs + f];
    yb -= mb[ML::S(1, 0) * vs + f];
  }
  // cell areas Omega = (d1 x d2)/2, d1 = P(a+1,b+1) - P(a,b), d2 = P(a,b+1) - P(a+1,b)
  for (int cb = j - 1; cb <= j; ++cb) {
    for (int ca = i - 1; ca <= i; ++ca) {
      if (ca < 0 || cb < 0 || ca >= B.ni || cb >= B.nj) continue;
      const double Ob = mb[ML::INVVOL * vs + pidx(B, ca, cb, 0)];
      const double d1x = X(0, ca + 1, cb + 1) - X(0, ca, cb), d1y = X(1, ca + 1, cb + 1) - X(1, ca, cb);
      const double d2x = X(0, ca, cb + 1) - X(0, ca + 1, cb), d2y = X(1, ca, cb + 1) - X(1, ca + 1, cb);
      // dOmega/dd1 = (d2y, -d2x)/2, dOmega/dd2 = (-d1y, d1x)/2
      if (ca == i && cb == j) {  // node is P(a,b): -d1
        xb -= 0.5 * Ob * d2y;
        yb += 0.5 * Ob * d2x;
      }
      if (ca == i - 1 && cb == j - 1) {  // node is P(a+1,b+1): +d1
        xb += 0.5 * Ob * d2y;
        yb -= 0.5 * Ob * d2x;
      }
      if (ca == i && cb == j - 1) {  // node is P(a,b+1): +d2
        xb -= 0.5 * Ob * d1y;
        yb += 0.5 * Ob * d1x;
      }
      if (ca == i - 1 && cb == j) {  // node is P(a+1,b): -d2
        xb += 0.5 * Ob * d1y;
        yb -= 0.5 * Ob * d1x;
      }
    }
  }
  Xb[0 * nn + B.node0 + c] = xb;
  Xb[1 * nn + B.node0 + c] = yb;
}

// ---------------------------------------------------------------------------
// cell sums (deterministic two-level reduction) and the uniform-state VJP

template <int DIM>
__global__ void __launch_bounds__(256) cell_sum_partial_kernel(const double* src, long long ncells, double* partial) {
  constexpr int NV = DIM + 2;
  __shared__ double red[256];
  const long long per = (ncells + gridDim.x - 1) / gridDim.x;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = min(ncells, lo + per);
  for (int v = 0; v < NV; ++v) {
    double s = 0.0;
    for (long long c = lo + threadIdx.x; c < hi; c += blockDim.x) s += src[v * ncells + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(long long)v * gridDim.x + blockIdx.x] = red[0];
    __syncthreads();
  }
}

// thetabar = (dQ/dq at theta)^T sum_cells Qbar
template <int DIM>
__global__ void uniform_state_vjp_kernel(const double* partial, int nparts, double* theta_io_bar, Gas g,
                                         double t0, double t1, double t2, double t3, double t4) {
  constexpr int NV = DIM + 2;
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double sb[NV];
  for (int v = 0; v < NV; ++v) {
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += partial[(long long)v * nparts + p];
    sb[v] = s;
  }
  const double th[5] = {t0, t1, t2, t3, t4};
  const double rho = th[0];
  double ke = 0.0;
  for (int d = 0; d < DIM; ++d) ke += th[1 + d] * th[1 + d];
  // Q = (rho, rho u, p/(g-1) + rho |u|^2 / 2)
  double out[NV];
  out[0] = sb[0] + sb[NV - 1] * 0.5 * ke;
  for (int d = 0; d < DIM; ++d) {
    out[0] += sb[1 + d] * th[1 + d];
    out[1 + d] = sb[1 + d] * rho + sb[NV - 1] * rho * th[1 + d];
  }
  out[NV - 1] = sb[NV - 1] * g.igm1;
  for (int v = 0; v < NV; ++v) theta_io_bar[v] = out[v];
}

// ---------------------------------------------------------------------------
// launchers

static dim3 grid2(long long n, int nb) { return dim3((unsigned)((n + 255) / 256), (unsigned)nb); }

#define DISPATCH_LIM(K, DIMV, ...)                                                                    \
  switch (lim) {                                                                                      \
    case LIM_NONE: hipLaunchKernelGGL((K<DIMV, LIM_NONE>), __VA_ARGS__); break;                     \
    case LIM_VANLEER: hipLaunchKernelGGL((K<DIMV, LIM_VANLEER>), __VA_ARGS__); break;               \
    default: hipLaunchKernelGGL((K<DIMV, LIM_VANALBADA>), __VA_ARGS__); break;                      \
  }

hipError_t launch_vjp_face(int dim, int lim, const VjpArgs& a, long long max_faces, int nb, hipStream_t s) {
  if (dim == 2) {
    DISPATCH_LIM(vjp_face_kernel, 2, grid2(max_faces, nb), dim3(256), 0, s, a)
  } else {
    DISPATCH_LIM(vjp_face_kernel, 3, grid2(max_faces, nb), dim3(256), 0, s, a)
  }
  return hipGetLastError();
}

hipError_t launch_vjp_cell(int dim, int lim, const VjpArgs& a, long long max_padded, int nb, hipStream_t s) {
  if (dim == 2) {
    DISPATCH_LIM(vjp_cell_kernel, 2, grid2(max_padded, nb), dim3(256), 0, s, a)
  } else {
    DISPATCH_LIM(vjp_cell_kernel, 3, grid2(max_padded, nb), dim3(256), 0, s, a)
  }
  return hipGetLastError();
}

hipError_t launch_vjp_ghost(int dim, const VjpArgs& a, const ChunkDev* chunks, int begin, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (dim == 2)
    hipLaunchKernelGGL(vjp_ghost_kernel<2>, dim3(count), dim3(CHUNK), 0, s, a, chunks, begin);
  else
    hipLaunchKernelGGL(vjp_ghost_kernel<3>, dim3(count), dim3(CHUNK), 0, s, a, chunks, begin);
  return hipGetLastError();
}

hipError_t launch_vjp_finalize(int dim, const VjpArgs& a, long long max_cells, int nb, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(vjp_finalize_kernel<2>, grid2(max_cells, nb), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(vjp_finalize_kernel<3>, grid2(max_cells, nb), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_vjp_inflow_reduce(int dim, const VjpArgs& a, const int* inflow_patches, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (dim == 2)
    hipLaunchKernelGGL(vjp_inflow_reduce_kernel<2>, dim3(n), dim3(256), 0, s, a, inflow_patches);
  else
    hipLaunchKernelGGL(vjp_inflow_reduce_kernel<3>, dim3(n), dim3(256), 0, s, a, inflow_patches);
  return hipGetLastError();
}

hipError_t launch_objective(int dim, const VjpArgs& a, const ChunkDev* chunks, int begin, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (dim == 2)
    hipLaunchKernelGGL(objective_kernel<2>, dim3(count), dim3(CHUNK), 0, s, a, chunks, begin);
  else
    hipLaunchKernelGGL(objective_kernel<3>, dim3(count), dim3(CHUNK), 0, s, a, chunks, begin);
  return hipGetLastError();
}

hipError_t launch_objective_sum(const VjpArgs& a, const int* wall_patches, int nwall, double* J, hipStream_t s) {
  hipLaunchKernelGGL(objective_sum_kernel, dim3(1), dim3(256), 0, s, a, wall_patches, nwall, J);
  return hipGetLastError();
}

hipError_t launch_node_vjp_2d(const VjpArgs& a, double* Xb, long long max_nodes, int nb, hipStream_t s) {
  hipLaunchKernelGGL(node_vjp_2d_kernel, grid2(max_nodes, nb), dim3(256), 0, s, a, Xb);
  return hipGetLastError();
}

hipError_t launch_uniform_state_vjp(int dim, const double* Qbar, long long ncells, double* partial, int nparts,
                                    double* thetabar, Gas g, const double* theta, hipStream_t s) {
  if (dim == 2) {
    hipLaunchKernelGGL(cell_sum_partial_kernel<2>, dim3(nparts), dim3(256), 0, s, Qbar, ncells, partial);
    hipLaunchKernelGGL(uniform_state_vjp_kernel<2>, dim3(1), dim3(64), 0, s, partial, nparts, thetabar, g, theta[0],
                       theta[1], theta[2], theta[3], theta[4]);
  } else {
    hipLaunchKernelGGL(cell_sum_partial_kernel<3>, dim3(nparts), dim3(256), 0, s, Qbar, ncells, partial);
    hipLaunchKernelGGL(uniform_state_vjp_kernel<3>, dim3(1), dim3(64), 0, s, partial, nparts, thetabar, g, theta[0],
                       theta[1], theta[2], theta[3], theta[4]);
  }
  return hipGetLastError();
}

}  // namespace cfd
