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
//      in 2D passes 1 and 2 run fused per tile with the face results in LDS;
//   3+4. gather-finalize: per interior cell, adds the cotangents of the ghost
//      cells filled from it (connections, mirror walls with their wall-normal
//      dJ/dS term, outflow copies), converts primitive to conservative
//      cotangents, and sums inflow ghost cotangents into dJ/dtheta.
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

// Qb = scale (dq/dQ)^T qb for interior cell (i,j,k); out = Qb; acc += Qb
template <int DIM>
__device__ void finalize_cell(const VjpArgs& a, const BlockDev& B, int i, int j, int k, const double* qv,
                              const double* qb) {
  constexpr int NV = DIM + 2;
  double Qb[NV];
  prim_cotangent_to_cons<DIM>(qv, qb, a.gas, Qb);
  const long long pc = B.packed + ((long long)k * B.nj + j) * B.ni + i;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double val = a.scale * Qb[v];
    if (a.out) a.out[v * B.ncell_total + pc] = val;
    if (a.acc) {
      double add = (a.acc_mode & 1) ? val : 0.0;
      if (a.acc_mode & 2) add = a.Rb[v * B.ncell_total + pc] + add;
      a.acc[v * B.ncell_total + pc] += add;
    }
  }
}

// true if cell (i,j,k) lies within NG layers of a face of its block
template <int DIM>
__device__ __forceinline__ bool near_face(const BlockDev& B, int i, int j, int k) {
  bool inner = i >= NG && i < B.ni - NG && j >= NG && j < B.nj - NG;
  if (DIM == 3) inner = inner && k >= NG && k < B.nk - NG;
  return !inner;
}

// 2D tile of TX x TY cells: true if every face within NG layers of interior
// cell (i,j) is covered by a physical patch (or nothing) at the cell's
// position and the tile holding the cell also holds that face's ghost cells
// (always on low faces; on high faces when the block ends inside the tile).
// codes[F] receives the face-map entries.
__device__ __forceinline__ void face_codes_2d(const VjpArgs& a, int b, const BlockDev& B, int i, int j, int* codes) {
#pragma unroll
  for (int F = 0; F < 4; ++F) {
    const int ax = F >> 1;
    const int x = ax == 0 ? i : j, n = ax == 0 ? B.ni : B.nj;
    const int g = (F & 1) ? n - 1 - x : x;
    codes[F] = g < NG ? a.facemap[a.fmap_off[b * 6 + F] + (ax == 0 ? j : i)] : FMAP_NONE;
  }
}

template <int TX, int TY>
__device__ __forceinline__ bool tile_physical_bc(const BlockDev& B, int i, int j, const int* codes) {
  const int i0 = i - i % TX, j0 = j - j % TY;
  bool ok = true;
#pragma unroll
  for (int F = 0; F < 4; ++F) {
    if (codes[F] == FMAP_NONE) continue;
    if (codes[F] >= 0) ok = false;
    if (F == 1 && i0 + TX < B.ni) ok = false;
    if (F == 3 && j0 + TY < B.nj) ok = false;
  }
  return ok;
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
  bool interior = true;
#pragma unroll
  for (int d = 0; d < DIM; ++d) interior = interior && co[d] >= 0 && co[d] < nn[d];
  if (interior && !near_face<DIM>(B, i, j, k)) {
    double qv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) qv[v] = q[v * vs];
    finalize_cell<DIM>(a, B, i, j, k, qv, qb);
  } else {
    double* out = a.qbar + B.origin + ci;
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v * vs] = qb[v];
  }
  if (interior) {
    // Omega-bar = -(1/Omega)-bar / Omega^2
    const double iv = a.metric[B.morigin + ML::INVVOL * vs + ci];
    a.metricbar[B.morigin + ML::INVVOL * vs + ci] += a.scale * (-ivb * iv * iv);
  }
}

// ---------------------------------------------------------------------------
// 1+2 fused (2D): per 16x16 tile, the face pass over every face whose state
// cotangents reach a cell of the tile (three-cell halo of q in LDS, faces on
// the tile edges recomputed by both neighbours, dJ/dS written by the tile
// that owns the face), then the cell pass from LDS: one slope VJP per cell
// and direction, gathered into the tile's cells and, on block edges, into
// the adjacent ghost cells.

template <int LIM, int TX, int TY>
__global__ void __launch_bounds__(TX* TY) vjp_tile2d_kernel(VjpArgs a) {
  constexpr int NV = 4, NT = TX * TY;
  constexpr int LX = TX + 6, LY = TY + 6;     // q of cells i0-3 .. i0+TX+2, j0-3 .. j0+TY+2
  constexpr int FXN = TX + 3, FYN = TY + 3;   // faces i0-1 .. i0+TX+1 (j0-1 .. j0+TY+1)
  constexpr int NFX = FXN * TY, NFY = TX * FYN;
  constexpr int NGH = 4 * TY + 4 * TX;        // ghost-cell items of a tile touching every block edge
  using ML = MetricLayout<2>;
  // LDS: q with halo, then the face results of both directions; the cell
  // phase later reuses the whole buffer for its per-cell arrays
  constexpr int NQ = NV * LX * LY, NFXA = (2 * NV + 3) * NFX, NFYA = (2 * NV + 3) * NFY;
  constexpr int NCELLA = (3 * NV + 1) * ((TX + 2) * TY + TX * (TY + 2));
  constexpr int NLDS = NQ + NFXA + NFYA > NCELLA ? NQ + NFXA + NFYA : NCELLA;
  __shared__ double lds[NLDS];
  auto sq = reinterpret_cast<double(*)[LX * LY]>(lds);
  auto fxL = reinterpret_cast<double(*)[NFX]>(lds + NQ);
  auto fxR = reinterpret_cast<double(*)[NFX]>(lds + NQ + NV * NFX);
  double* fxP = lds + NQ + 2 * NV * NFX;
  double* fxCL = fxP + NFX;
  double* fxCR = fxCL + NFX;
  auto fyL = reinterpret_cast<double(*)[NFY]>(lds + NQ + NFXA);
  auto fyR = reinterpret_cast<double(*)[NFY]>(lds + NQ + NFXA + NV * NFY);
  double* fyP = lds + NQ + NFXA + 2 * NV * NFY;
  double* fyCL = fyP + NFY;
  double* fyCR = fyCL + NFY;

  const int tid = threadIdx.x;
  // rank of this lane in the face and cell-item rounds: the last, partial
  // round of each falls on a few waves, which rotate from tile to tile so the
  // extra work does not always land on the same SIMD
  static_assert(NT % 64 == 0, "whole wavefronts per workgroup");
  const int rt = (tid + 64 * (int)(blockIdx.x % (NT / 64))) % NT;
  const TileDev tile = a.vtiles[blockIdx.x];
  const int b = tile.block;
  const BlockDev B = a.blocks[b];
  const int i0 = tile.i0, j0 = tile.j0;
  const long long vs = B.vstride;
  const double* q = a.q + B.origin;
  const double* met = a.metric + B.morigin;
  // face-map entries of the thread's tile cell (used by its boundary transposes)
  int codes[4];
  face_codes_2d(a, b, B, min(i0 + tid % TX, B.ni - 1), min(j0 + tid / TX, B.nj - 1), codes);

  for (int e = tid; e < LX * LY; e += NT) {
    const int i = i0 - 3 + e % LX, j = j0 - 3 + e / LX;
    if (i >= -2 && i <= B.ni + 1 && j >= -2 && j <= B.nj + 1) {
      const long long p = pidx(B, i, j, 0);
#pragma unroll
      for (int v = 0; v < NV; ++v) sq[v][e] = q[v * vs + p];
    }
  }
  __syncthreads();

  // ---- faces
  for (int e = rt; e < NFX + NFY; e += NT) {
    const int d = e < NFX ? 0 : 1;
    int f, t, slot, lc, st;
    if (d == 0) {
      const int r = e / FXN, fi = e % FXN;
      f = i0 - 1 + fi;
      t = j0 + r;
      slot = e;
      lc = (r + 3) * LX + fi + 2;  // cell f (right of the face)
      st = 1;
    } else {
      const int e2 = e - NFX, fj = e2 / TX, c = e2 % TX;
      f = j0 - 1 + fj;
      t = i0 + c;
      slot = e2;
      lc = (fj + 2) * LX + c + 3;
      st = LX;
    }
    const int n = d == 0 ? B.ni : B.nj, nt = d == 0 ? B.nj : B.ni;
    double Lb[NV], Rb_[NV], F[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Lb[v] = Rb_[v] = F[v] = 0.0;
    double P = 0.0, cL = 0.0, cR = 0.0;
    if (f >= 0 && f <= n && t >= 0 && t < nt) {
      const int iR = d == 0 ? f : t, jR = d == 0 ? t : f;
      const long long fidx = pidx(B, iR, jR, 0);
      const long long step = d == 0 ? 1LL : (long long)B.pi;
      double S[2], Sb[2] = {0.0, 0.0};
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) S[cc] = met[ML::S(d, cc) * vs + fidx];
      const bool Lin = f >= 1, Rin = f < n;
      const long long pcR = B.packed + (long long)jR * B.ni + iR;
      const long long pcL = pcR - (d == 0 ? 1LL : (long long)B.ni);
      const double ivL = Lin ? met[ML::INVVOL * vs + fidx - step] : 0.0;
      const double ivR = Rin ? met[ML::INVVOL * vs + fidx] : 0.0;
      double Fb[NV], RbL[NV], RbR[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        RbL[v] = Lin ? a.Rb[v * B.ncell_total + pcL] : 0.0;
        RbR[v] = Rin ? a.Rb[v * B.ncell_total + pcR] : 0.0;
        Fb[v] = RbL[v] * ivL - RbR[v] * ivR;
      }
      const int face = f == 0 ? 2 * d : (f == n ? 2 * d + 1 : -1);
      if (face >= 0 && (B.wall_mask & (1 << face)) && wall_at(a, b, face, t, 0)) {
        const double p0 = (face & 1) ? sq[NV - 1][lc - st] : sq[NV - 1][lc];
        const double p1 = (face & 1) ? sq[NV - 1][lc - 2 * st] : sq[NV - 1][lc + st];
        const double pw = 1.5 * p0 - 0.5 * p1;
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
          F[1 + cc] = pw * S[cc];
          P += Fb[1 + cc] * S[cc];
          Sb[cc] += pw * Fb[1 + cc];
        }
      } else {
        double qL[NV], qR[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double qm = sq[v][lc - 2 * st], qa = sq[v][lc - st], qb = sq[v][lc], qp = sq[v][lc + st];
          double spa, sma, spb, smb;
          cell_slopes<LIM>(qa - qm, qb - qa, a.e2[v], a.kappa, spa, sma);
          cell_slopes<LIM>(qb - qa, qp - qb, a.e2[v], a.kappa, spb, smb);
          qL[v] = qa + a.half_eps * spa;
          qR[v] = qb - a.half_eps * smb;
        }
        roe_flux_vjp<2>(qL, qR, S, a.gas, a.efix, a.half_inv_efix, Fb, F, Lb, Rb_, Sb);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        cL += RbL[v] * F[v];
        cR -= RbR[v] * F[v];
      }
      // dJ/dS by the tile holding cell min(f, n-1)
      const int own0 = d == 0 ? i0 : j0, town = d == 0 ? TX : TY;
      const int fo = f < n ? f : n - 1;
      if (fo >= own0 && fo < own0 + town) {
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) a.metricbar[B.morigin + ML::S(d, cc) * vs + fidx] += a.scale * Sb[cc];
      }
    }
    if (d == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        fxL[v][slot] = Lb[v];
        fxR[v][slot] = Rb_[v];
      }
      fxP[slot] = P;
      fxCL[slot] = cL;
      fxCR[slot] = cR;
    } else {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        fyL[v][slot] = Lb[v];
        fyR[v][slot] = Rb_[v];
      }
      fyP[slot] = P;
      fyCL[slot] = cL;
      fyCR[slot] = cR;
    }
  }
  __syncthreads();

  // ---- per cell m along each direction (m = o-1 .. o+T): the slope cotangent
  // split (G = cotangent of q_{m+1} - q_m, H = of q_m - q_{m-1}), the cell's
  // own terms Own = Lbar(m+1) + Rbar(m) + H - G (+ wall pressure terms), and
  // the 1/Omega cotangent; then q-bar_x = sum_d Own_x + G_{x-1} - H_{x+1}.
  constexpr int NCX = (TX + 2) * TY, NCY = TX * (TY + 2);
  constexpr int NCI = NCX + NCY;
  constexpr int RPT = (NCI + NT - 1) / NT;  // items per thread
  double rOwn[RPT][NV], rG[RPT][NV], rH[RPT][NV], rI[RPT];
  double qown[NV];  // q of this thread's tile cell (the LDS copy is reused below)
#pragma unroll
  for (int v = 0; v < NV; ++v) qown[v] = sq[v][(tid / TX + 3) * LX + tid % TX + 3];
#pragma unroll
  for (int it = 0; it < RPT; ++it) {
    const int e = rt + it * NT;
#pragma unroll
    for (int v = 0; v < NV; ++v) rOwn[it][v] = rG[it][v] = rH[it][v] = 0.0;
    rI[it] = 0.0;
    if (e >= NCI) continue;
    const int d = e < NCX ? 0 : 1;
    int r, m;
    if (d == 0) {
      r = e / (TX + 2);
      m = i0 - 1 + e % (TX + 2);
    } else {
      const int e2 = e - NCX;
      r = e2 % TX;
      m = j0 - 1 + e2 / TX;
    }
    const int n = d == 0 ? B.ni : B.nj, nt = d == 0 ? B.nj : B.ni;
    const int o = d == 0 ? i0 : j0;
    const int t = (d == 0 ? j0 : i0) + r;
    if (t < 0 || t >= nt || m < -1 || m > n) continue;
    const double* FL = d == 0 ? &fxL[0][0] : &fyL[0][0];
    const double* FR = d == 0 ? &fxR[0][0] : &fyR[0][0];
    const int fstride = d == 0 ? NFX : NFY;
    auto fslot = [&](int f) { return d == 0 ? r * FXN + (f - o + 1) : (f - o + 1) * TX + r; };
    auto cpos = [&](int x) { return d == 0 ? (r + 3) * LX + (x - o + 3) : (x - o + 3) * LX + r + 3; };
    const bool hp = m + 1 <= n;  // face m+1 exists
    const bool hm = m >= 0;      // face m exists
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double lb = hp ? FL[v * fstride + fslot(m + 1)] : 0.0;
      const double rb = hm ? FR[v * fstride + fslot(m)] : 0.0;
      const double spb = a.half_eps * lb, smb = -a.half_eps * rb;
      double gp = 0.0, hmv = 0.0;
      if (spb != 0.0 || smb != 0.0) {
        const double qm1 = sq[v][cpos(m - 1)], q0 = sq[v][cpos(m)], qp1 = sq[v][cpos(m + 1)];
        slope_vjp<LIM>(q0 - qm1, qp1 - q0, a.e2[v], a.kappa, spb, smb, gp, hmv);
      }
      rG[it][v] = gp;
      rH[it][v] = hmv;
      rOwn[it][v] = (lb + rb) + (hmv - gp);
    }
    if (m >= 0 && m < n) {
      if (B.wall_mask & (3 << (2 * d))) {
        // wall pressure extrapolation p_w = 1.5 p0 - 0.5 p1 on wall faces 0 and n
        // (the pressure cotangent of a face is zero unless it is a wall face)
        // (face n lies outside this tile's face range only for a cell m = o+T,
        // whose own terms no cell of the tile uses)
        const double* FP = d == 0 ? fxP : fyP;
        const int nf = d == 0 ? FXN : FYN;
        if (m == 0 || m == 1) rOwn[it][NV - 1] += (m == 0 ? 1.5 : -0.5) * FP[fslot(0)];
        if ((m == n - 1 || m == n - 2) && n - o + 1 < nf)
          rOwn[it][NV - 1] += (m == n - 1 ? 1.5 : -0.5) * FP[fslot(n)];
      }
      const double* CL = d == 0 ? fxCL : fyCL;
      const double* CR = d == 0 ? fxCR : fyCR;
      rI[it] = CL[fslot(m + 1)] + CR[fslot(m)];
    }
  }
  __syncthreads();
  // the per-cell arrays reuse the LDS of q and of the face arrays
  double* cOwn = lds;                  // [NV][NCI]
  double* cG = cOwn + NV * NCI;        // [NV][NCI]
  double* cH = cG + NV * NCI;          // [NV][NCI]
  double* cI = cH + NV * NCI;          // [NCI]
#pragma unroll
  for (int it = 0; it < RPT; ++it) {
    const int e = rt + it * NT;
    if (e >= NCI) continue;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      cOwn[v * NCI + e] = rOwn[it][v];
      cG[v * NCI + e] = rG[it][v];
      cH[v * NCI + e] = rH[it][v];
    }
    cI[e] = rI[it];
  }
  __syncthreads();

  // ---- q-bar of the tile's cells, then of ghost cells on block edges.  A cell
  // whose ghost copies all belong to physical patches of faces whose ghost
  // cells this tile computes is finalized here (after the barrier below); a
  // cell next to a connection is left to vjp_boundary_gather_kernel.
  double* gq = lds + NCELLA;  // [NV][NGH] ghost q-bar of this tile
  static_assert(NCELLA + NV * NGH <= NLDS, "LDS too small for the ghost q-bar");
  const bool lo_i = i0 == 0, hi_i = i0 + TX >= B.ni, lo_j = j0 == 0, hi_j = j0 + TY >= B.nj;
  double qdef[NV];
  bool deferred = false;
  for (int e = tid; e < NT + NGH; e += NT) {
    int i, j;
    bool ok;
    if (e < NT) {
      i = i0 + e % TX;
      j = j0 + e / TX;
      ok = i < B.ni && j < B.nj;
    } else {
      const int g = e - NT;
      const int layer = g & 1, pos = (g >> 1);
      if (g < 4 * TY) {  // i-ghosts of the tile's rows: low side, then high side
        const bool hi = g >= 2 * TY;
        j = j0 + (pos % TY);
        i = hi ? B.ni + layer : -1 - layer;
        ok = (hi ? hi_i : lo_i) && j < B.nj;
      } else {  // j-ghosts of the tile's columns
        const int g2 = g - 4 * TY, pos2 = g2 >> 1;
        const bool hi = g2 >= 2 * TX;
        i = i0 + (pos2 % TX);
        j = hi ? B.nj + layer : -1 - layer;
        ok = (hi ? hi_j : lo_j) && i < B.ni;
      }
    }
    if (!ok) continue;
    double qbv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) qbv[v] = 0.0;
    double ivb = 0.0;
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const bool others_in = d == 0 ? (j >= 0 && j < B.nj) : (i >= 0 && i < B.ni);
      if (!others_in) continue;
      const int x = d == 0 ? i : j;
      const int o = d == 0 ? i0 : j0;
      const int T = d == 0 ? TX : TY;
      const int r = d == 0 ? j - j0 : i - i0;
      // cell-array index of cell m along d (valid for o-1 <= m <= o+T)
      auto cidx = [&](int m) { return d == 0 ? r * (TX + 2) + (m - o + 1) : NCX + (m - o + 1) * TX + r; };
      const bool in0 = x >= o - 1 && x <= o + T;
      const bool inm = x - 1 >= o - 1 && x - 1 <= o + T;
      const bool inp = x + 1 >= o - 1 && x + 1 <= o + T;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double own = in0 ? cOwn[v * NCI + cidx(x)] : 0.0;
        const double gl = inm ? cG[v * NCI + cidx(x - 1)] : 0.0;
        const double hr = inp ? cH[v * NCI + cidx(x + 1)] : 0.0;
        qbv[v] += own + (gl - hr);
      }
      if (in0) ivb += cI[cidx(x)];
    }
    const long long ci = pidx(B, i, j, 0);
    const bool interior = i >= 0 && i < B.ni && j >= 0 && j < B.nj;
    bool to_global = true;
    if (e >= NT) {
#pragma unroll
      for (int v = 0; v < NV; ++v) gq[v * NGH + (e - NT)] = qbv[v];
    } else if (interior && !near_face<2>(B, i, j, 0)) {
      finalize_cell<2>(a, B, i, j, 0, qown, qbv);  // e == tid here: the thread's tile cell
      to_global = false;
    } else if (interior && tile_physical_bc<TX, TY>(B, i, j, codes)) {
#pragma unroll
      for (int v = 0; v < NV; ++v) qdef[v] = qbv[v];
      deferred = true;
      to_global = false;
    }
    if (to_global) {
      double* out = a.qbar + B.origin + ci;
#pragma unroll
      for (int v = 0; v < NV; ++v) out[v * vs] = qbv[v];
    }
    if (interior) {
      const double iv = met[ML::INVVOL * vs + ci];
      a.metricbar[B.morigin + ML::INVVOL * vs + ci] += a.scale * (-ivb * iv * iv);
    }
  }
  __syncthreads();
  if (deferred) {
    // the thread's tile cell: physical-patch transposes from the ghost q-bar in LDS
    const int i = i0 + tid % TX, j = j0 + tid / TX;
    auto ghost_item = [&](int F, int gl) {
      return F == 0 ? 2 * (j - j0) + gl
                    : (F == 1 ? 2 * TY + 2 * (j - j0) + gl
                              : (F == 2 ? 4 * TY + 2 * (i - i0) + gl : 4 * TY + 2 * TX + 2 * (i - i0) + gl));
    };
    for (int F = 0; F < 4; ++F) {
      const int ax = F >> 1;
      const bool hi = F & 1;
      const int x = ax == 0 ? i : j, n = ax == 0 ? B.ni : B.nj;
      const int g = hi ? n - 1 - x : x;
      if (g >= NG || codes[F] == FMAP_NONE) continue;
      const int pid = -codes[F] - 1;
      const PatchDev p = a.patches[pid];
      const int t1 = ax == 0 ? j : i;
      if (p.kind == PK_EXTRAP_OUTFLOW) {
        if (g != 0) continue;
        for (int gl = 0; gl < NG; ++gl) {
#pragma unroll
          for (int v = 0; v < NV; ++v) qdef[v] += gq[v * NGH + ghost_item(F, gl)];
        }
      } else if (p.kind == PK_SUP_INFLOW) {
        if (g != 0) continue;
        double sacc[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) sacc[v] = 0.0;
        for (int gl = 0; gl < NG; ++gl) {
#pragma unroll
          for (int v = 0; v < NV; ++v) sacc[v] += gq[v * NGH + ghost_item(F, gl)];
        }
        const int cnt = p.len0 * p.len1;
        const int e = t1 - p.lo0;
        double* part = a.inflow_part + a.part_offset[pid];
#pragma unroll
        for (int v = 0; v < NV; ++v) part[v * cnt + e] += a.scale * sacc[v];
      } else {
        // slip wall: ghost layer gl mirrors interior layer gl about the face
        int fi, fj, fk;
        face_cell(B, 2, F, 0, hi, t1, 0, fi, fj, fk);
        const long long fidx = pidx(B, fi, fj, fk);
        double S[2], Sb[2] = {0.0, 0.0};
        double s2 = 0.0;
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
          S[cc] = met[ML::S(ax, cc) * vs + fidx];
          s2 += S[cc] * S[cc];
        }
        const double is2 = 1.0 / s2;
        for (int gl = 0; gl < NG; ++gl) {
          if (gl != g && g != 0) continue;  // the cell next to the wall also forms dJ/dS of both layers
          int mi, mj, mk;
          face_cell(B, 2, F, gl, false, t1, 0, mi, mj, mk);
          const long long midx = pidx(B, mi, mj, mk);
          const int gi_ = ghost_item(F, gl);
          double ug[2], um[2];
          double un = 0.0, ugS = 0.0;
#pragma unroll
          for (int cc = 0; cc < 2; ++cc) {
            ug[cc] = gq[(1 + cc) * NGH + gi_];
            um[cc] = gl == g ? qown[1 + cc] : q[(1 + cc) * vs + midx];
            un += um[cc] * S[cc];
            ugS += ug[cc] * S[cc];
          }
          if (gl == g) {
            qdef[0] += gq[gi_];
            qdef[NV - 1] += gq[(NV - 1) * NGH + gi_];
#pragma unroll
            for (int cc = 0; cc < 2; ++cc) qdef[1 + cc] += ug[cc] - 2.0 * ugS * S[cc] * is2;
          }
          if (g == 0) {
            const double fco = 2.0 * un * is2;
#pragma unroll
            for (int cc = 0; cc < 2; ++cc)
              Sb[cc] += -fco * ug[cc] - ugS * (2.0 * um[cc] * is2 - 4.0 * un * S[cc] * is2 * is2);
          }
        }
        if (g == 0) {
#pragma unroll
          for (int cc = 0; cc < 2; ++cc) a.metricbar[B.morigin + ML::S(ax, cc) * vs + fidx] += a.scale * Sb[cc];
        }
      }
    }
    finalize_cell<2>(a, B, i, j, 0, qown, qdef);
  }
}

// ---------------------------------------------------------------------------
// 3+4 gather and finalize of one interior cell: add the cotangents of the
// ghost cells that copy it (connections: the receiving block's ghost;
// outflow: both ghost layers into the adjacent cell; slip wall: the mirrored
// ghost, with the wall-normal term of dJ/dS taken by the cell next to the
// wall), faces in order 0 .. 2 dim - 1, then Qb = scale (dq/dQ)^T qb;
// out = Qb; acc += Qb.  Cells next to inflow faces add scale times the sum of
// the inflow ghost cotangents at their position to that patch's partial sums
// (reduced into dJ/dtheta by vjp_inflow_reduce_kernel).  Only cells within
// NG layers of a face receive ghost cotangents; the pass kernels finalize
// every other interior cell themselves.

template <int DIM>
__device__ void gather_finalize_cell(const VjpArgs& a, int b, const BlockDev& B, int i, int j, int k) {
  constexpr int NV = DIM + 2;
  using ML = MetricLayout<DIM>;
  const long long vs = B.vstride;
  const long long ci = pidx(B, i, j, k);
  double* qbb = a.qbar + B.origin;
  double qb[NV], qv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    qb[v] = qbb[v * vs + ci];
    qv[v] = a.q[B.origin + v * vs + ci];
  }
  const int co[3] = {i, j, k};
  const int nn[3] = {B.ni, B.nj, B.nk};
  for (int F = 0; F < 2 * DIM; ++F) {
    const int ax = F >> 1;
    const bool hi = F & 1;
    const int g = hi ? nn[ax] - 1 - co[ax] : co[ax];
    if (g >= NG) continue;
    int t1, t2;
    tang(ax, i, j, k, t1, t2);
    const int T1 = ax == 0 ? B.nj : B.ni;
    const int code = a.facemap[a.fmap_off[b * 6 + F] + t1 + (long long)t2 * T1];
    if (code >= 0) {
      const TransferDev x = a.xfers[code];
      // inverse of orient_map: donor offset -> receiver offset
      const int d1 = t1 - x.dlo0, d2 = t2 - x.dlo1;
      const int s1 = (x.orient & 1) ? x.dlen0 - 1 - d1 : d1;
      const int s2 = (x.orient & 2) ? x.dlen1 - 1 - d2 : d2;
      const int r1 = (x.orient & 4) ? s2 : s1, r2 = (x.orient & 4) ? s1 : s2;
      const BlockDev& R = a.blocks[x.rblock];
      int gi, gj, gk;
      face_cell(R, DIM, x.rface, g, true, x.rlo0 + r1, x.rlo1 + r2, gi, gj, gk);
      const double* src = a.qbar + R.origin + pidx(R, gi, gj, gk);
#pragma unroll
      for (int v = 0; v < NV; ++v) qb[v] += src[v * R.vstride];
      continue;
    }
    if (code == FMAP_NONE) continue;
    const int pid = -code - 1;
    const PatchDev p = a.patches[pid];
    if (p.kind == PK_EXTRAP_OUTFLOW) {
      if (g != 0) continue;
      for (int gl = 0; gl < NG; ++gl) {
        int gi, gj, gk;
        face_cell(B, DIM, F, gl, true, t1, t2, gi, gj, gk);
        const long long gidx = pidx(B, gi, gj, gk);
#pragma unroll
        for (int v = 0; v < NV; ++v) qb[v] += qbb[v * vs + gidx];
      }
    } else if (p.kind == PK_SUP_INFLOW) {
      if (g != 0) continue;
      double s[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) s[v] = 0.0;
      for (int gl = 0; gl < NG; ++gl) {
        int gi, gj, gk;
        face_cell(B, DIM, F, gl, true, t1, t2, gi, gj, gk);
        const long long gidx = pidx(B, gi, gj, gk);
#pragma unroll
        for (int v = 0; v < NV; ++v) s[v] += qbb[v * vs + gidx];
      }
      const int cnt = p.len0 * p.len1;
      const int e = (t1 - p.lo0) + (t2 - p.lo1) * p.len0;
      double* part = a.inflow_part + a.part_offset[pid];
#pragma unroll
      for (int v = 0; v < NV; ++v) part[v * cnt + e] += a.scale * s[v];
    } else {
      // slip wall: ghost layer g is the mirror of interior layer g about the face
      int fi, fj, fk;
      face_cell(B, DIM, F, 0, hi, t1, t2, fi, fj, fk);
      const long long fidx = pidx(B, fi, fj, fk);
      double S[DIM], Sb[DIM];
      double s2 = 0.0;
#pragma unroll
      for (int cc = 0; cc < DIM; ++cc) {
        S[cc] = a.metric[B.morigin + ML::S(ax, cc) * vs + fidx];
        s2 += S[cc] * S[cc];
        Sb[cc] = 0.0;
      }
      const double is2 = 1.0 / s2;
      for (int gl = 0; gl < NG; ++gl) {
        if (gl != g && g != 0) continue;  // the cell next to the wall also forms dJ/dS of both layers
        int gi, gj, gk, mi, mj, mk;
        face_cell(B, DIM, F, gl, true, t1, t2, gi, gj, gk);
        face_cell(B, DIM, F, gl, false, t1, t2, mi, mj, mk);
        const long long gidx = pidx(B, gi, gj, gk), midx = pidx(B, mi, mj, mk);
        double ug[DIM], um[DIM];
        double un = 0.0, ugS = 0.0;
#pragma unroll
        for (int cc = 0; cc < DIM; ++cc) {
          ug[cc] = qbb[(1 + cc) * vs + gidx];
          um[cc] = a.q[B.origin + (1 + cc) * vs + midx];
          un += um[cc] * S[cc];
          ugS += ug[cc] * S[cc];
        }
        if (gl == g) {
          qb[0] += qbb[gidx];
          qb[NV - 1] += qbb[(NV - 1) * vs + gidx];
#pragma unroll
          for (int cc = 0; cc < DIM; ++cc) qb[1 + cc] += ug[cc] - 2.0 * ugS * S[cc] * is2;
        }
        if (g == 0) {
          const double fco = 2.0 * un * is2;
#pragma unroll
          for (int cc = 0; cc < DIM; ++cc)
            Sb[cc] += -fco * ug[cc] - ugS * (2.0 * um[cc] * is2 - 4.0 * un * S[cc] * is2 * is2);
        }
      }
      if (g == 0) {
#pragma unroll
        for (int cc = 0; cc < DIM; ++cc) a.metricbar[B.morigin + ML::S(ax, cc) * vs + fidx] += a.scale * Sb[cc];
      }
    }
  }
  finalize_cell<DIM>(a, B, i, j, k, qv, qb);
}

// one thread per (block, face, layer < NG, tangential position); a cell near
// several faces is taken by the lowest of them
template <int DIM>
__global__ void __launch_bounds__(256) vjp_boundary_gather_kernel(VjpArgs a) {
  constexpr int NF = 2 * DIM;
  const int b = blockIdx.y / NF, F = blockIdx.y % NF;
  const BlockDev B = a.blocks[b];
  const int ax = F >> 1;
  const int T1 = ax == 0 ? B.nj : B.ni;
  const int T2 = DIM == 3 ? (ax == 2 ? B.nj : B.nk) : 1;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long area = (long long)T1 * T2;
  if (e >= NG * area) return;
  const int layer = (int)(e / area);
  const int t1 = (int)(e % area % T1), t2 = (int)(e % area / T1);
  const int nax = ax == 0 ? B.ni : (ax == 1 ? B.nj : B.nk);
  if (layer >= nax) return;
  int i, j, k;
  face_cell(B, DIM, F, layer, false, t1, t2, i, j, k);
  const int co[3] = {i, j, k};
  const int nn[3] = {B.ni, B.nj, B.nk};
  for (int G = 0; G < F; ++G) {
    const int g = (G & 1) ? nn[G >> 1] - 1 - co[G >> 1] : co[G >> 1];
    if (g < NG) return;
  }
  if (DIM == 2 && a.tile_bc) {
    int codes[4];
    face_codes_2d(a, b, B, i, j, codes);
    if (tile_physical_bc<VJP_TILE, VJP_TILE>(B, i, j, codes)) return;  // finalized by the tile pass
  }
  gather_finalize_cell<DIM>(a, b, B, i, j, k);
}

// inflow partial sums -> theta-bar (one workgroup per inflow patch, fixed order)
template <int DIM>
__global__ void __launch_bounds__(256) vjp_inflow_reduce_kernel(VjpArgs a) {
  constexpr int NV = DIM + 2;
  __shared__ double red[256];
  const int pid = a.inflow_list[blockIdx.x];
  const PatchDev p = a.patches[pid];
  const int cnt = p.len0 * p.len1;
  const double* part = a.inflow_part + a.part_offset[pid];
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
// finalize alone (objective gradient): Qb = scale * (dq/dQ)^T qb ; out = Qb ; acc += Qb

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
// node gradient (3D): gather dJ/dS and dJ/dOmega onto the nodes
//
// A face with nodes a b c d has S = 1/2 (c - a) x (d - b) and mean node
// m = (a + b + c + d) / 4; a cell volume is 1/3 of the sum over its faces of
// m . S with outward sign, so face f along an axis (high face of cell f-1, low
// face of cell f) passes w = (Ob(f-1) - Ob(f)) / 3 to d(m . S).  With
// St = Sb + w m, u = c - a and v = d - b:  ubar = 1/2 v x St and
// vbar = 1/2 St x u; a takes -ubar, c +ubar, b -vbar, d +vbar, and each of
// the four nodes w S / 4.  One thread per node gathers its (up to) twelve faces.

__device__ __forceinline__ void cross3v(const double* x, const double* y, double* z) {
  z[0] = x[1] * y[2] - x[2] * y[1];
  z[1] = x[2] * y[0] - x[0] * y[2];
  z[2] = x[0] * y[1] - x[1] * y[0];
}

__global__ void __launch_bounds__(256) node_vjp_3d_kernel(VjpArgs a, double* Xb) {
  using ML = MetricLayout<3>;
  const BlockDev B = a.blocks[blockIdx.y];
  const int ni1 = B.ni + 1, nj1 = B.nj + 1, nk1 = B.nk + 1;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long long)ni1 * nj1 * nk1) return;
  const int node[3] = {(int)(c % ni1), (int)((c / ni1) % nj1), (int)(c / ((long long)ni1 * nj1))};
  const int n[3] = {B.ni, B.nj, B.nk};
  const long long vs = B.vstride, nn = B.nnode_total;
  const double* mb = a.metricbar + B.morigin;
  // corner offsets of a, b, c, d per face axis (the node order of the forward metrics)
  constexpr int OFF[3][4][3] = {{{0, 0, 0}, {0, 1, 0}, {0, 1, 1}, {0, 0, 1}},
                                {{0, 0, 0}, {0, 0, 1}, {1, 0, 1}, {1, 0, 0}},
                                {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0}}};
  double xb[3] = {0.0, 0.0, 0.0};
  for (int ax = 0; ax < 3; ++ax) {
    for (int r = 0; r < 4; ++r) {
      int f[3];
      bool ok = true;
      for (int d = 0; d < 3; ++d) {
        f[d] = node[d] - OFF[ax][r][d];
        if (d != ax && (f[d] < 0 || f[d] >= n[d])) ok = false;
      }
      if (!ok) continue;
      double p[4][3];
      for (int q = 0; q < 4; ++q) {
        const long long o =
            B.node0 + ((long long)(f[2] + OFF[ax][q][2]) * nj1 + f[1] + OFF[ax][q][1]) * ni1 + f[0] + OFF[ax][q][0];
        for (int cc = 0; cc < 3; ++cc) p[q][cc] = a.nodes[cc * nn + o];
      }
      double u[3], v[3], m[3], S[3], St[3];
      for (int cc = 0; cc < 3; ++cc) {
        u[cc] = p[2][cc] - p[0][cc];
        v[cc] = p[3][cc] - p[1][cc];
        m[cc] = 0.25 * (p[0][cc] + p[1][cc] + p[2][cc] + p[3][cc]);
      }
      cross3v(u, v, S);
      for (int cc = 0; cc < 3; ++cc) S[cc] *= 0.5;
      // w = (Ob(f-1) - Ob(f)) / 3 along the face axis; cells outside the block give 0
      double w = 0.0;
      if (f[ax] > 0) {
        int g[3] = {f[0], f[1], f[2]};
        g[ax] -= 1;
        w += mb[ML::INVVOL * vs + pidx(B, g[0], g[1], g[2])];
      }
      if (f[ax] < n[ax]) w -= mb[ML::INVVOL * vs + pidx(B, f[0], f[1], f[2])];
      w *= (1.0 / 3.0);
      const long long fidx = pidx(B, f[0], f[1], f[2]);
      for (int cc = 0; cc < 3; ++cc) St[cc] = mb[ML::S(ax, cc) * vs + fidx] + w * m[cc];
      double g[3];
      if (r == 0 || r == 2) {
        cross3v(v, St, g);  // 2 ubar
        const double sg = r == 0 ? -0.5 : 0.5;
        for (int cc = 0; cc < 3; ++cc) xb[cc] += sg * g[cc];
      } else {
        cross3v(St, u, g);  // 2 vbar
        const double sg = r == 1 ? -0.5 : 0.5;
        for (int cc = 0; cc < 3; ++cc) xb[cc] += sg * g[cc];
      }
      for (int cc = 0; cc < 3; ++cc) xb[cc] += 0.25 * w * S[cc];
    }
  }
  for (int cc = 0; cc < 3; ++cc) Xb[cc * nn + B.node0 + c] = xb[cc];
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
  __shared__ double red[256];
  double sb[NV];
  for (int v = 0; v < NV; ++v) {
    double s = 0.0;
    for (int p = threadIdx.x; p < nparts; p += blockDim.x) s += partial[(long long)v * nparts + p];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    sb[v] = red[0];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
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

hipError_t launch_vjp_tile2d(int lim, const VjpArgs& a, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  constexpr int T = VJP_TILE;
  switch (lim) {
    case LIM_NONE: hipLaunchKernelGGL((vjp_tile2d_kernel<LIM_NONE, T, T>), dim3(ntiles), dim3(T * T), 0, s, a); break;
    case LIM_VANLEER:
      hipLaunchKernelGGL((vjp_tile2d_kernel<LIM_VANLEER, T, T>), dim3(ntiles), dim3(T * T), 0, s, a);
      break;
    default:
      hipLaunchKernelGGL((vjp_tile2d_kernel<LIM_VANALBADA, T, T>), dim3(ntiles), dim3(T * T), 0, s, a);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_vjp_boundary_gather(int dim, const VjpArgs& a, long long max_face_area, int nb, hipStream_t s) {
  const dim3 grid((unsigned)((NG * max_face_area + 255) / 256), (unsigned)(nb * 2 * dim));
  if (dim == 2)
    hipLaunchKernelGGL(vjp_boundary_gather_kernel<2>, grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(vjp_boundary_gather_kernel<3>, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_vjp_inflow_reduce(int dim, const VjpArgs& a, hipStream_t s) {
  if (a.ninflow <= 0) return hipSuccess;
  if (dim == 2)
    hipLaunchKernelGGL(vjp_inflow_reduce_kernel<2>, dim3(a.ninflow), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(vjp_inflow_reduce_kernel<3>, dim3(a.ninflow), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_vjp_finalize(int dim, const VjpArgs& a, long long max_cells, int nb, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(vjp_finalize_kernel<2>, grid2(max_cells, nb), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(vjp_finalize_kernel<3>, grid2(max_cells, nb), dim3(256), 0, s, a);
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

hipError_t launch_node_vjp(int dim, const VjpArgs& a, double* Xb, long long max_nodes, int nb, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(node_vjp_2d_kernel, grid2(max_nodes, nb), dim3(256), 0, s, a, Xb);
  else
    hipLaunchKernelGGL(node_vjp_3d_kernel, grid2(max_nodes, nb), dim3(256), 0, s, a, Xb);
  return hipGetLastError();
}

hipError_t launch_uniform_state_vjp(int dim, const double* Qbar, long long ncells, double* partial, int nparts,
                                    double* thetabar, Gas g, const double* theta, hipStream_t s) {
  if (dim == 2) {
    hipLaunchKernelGGL(cell_sum_partial_kernel<2>, dim3(nparts), dim3(256), 0, s, Qbar, ncells, partial);
    hipLaunchKernelGGL(uniform_state_vjp_kernel<2>, dim3(1), dim3(256), 0, s, partial, nparts, thetabar, g, theta[0],
                       theta[1], theta[2], theta[3], theta[4]);
  } else {
    hipLaunchKernelGGL(cell_sum_partial_kernel<3>, dim3(nparts), dim3(256), 0, s, Qbar, ncells, partial);
    hipLaunchKernelGGL(uniform_state_vjp_kernel<3>, dim3(1), dim3(256), 0, s, partial, nparts, thetabar, g, theta[0],
                       theta[1], theta[2], theta[3], theta[4]);
  }
  return hipGetLastError();
}

}  // namespace cfd
