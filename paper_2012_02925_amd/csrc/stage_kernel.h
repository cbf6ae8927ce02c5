// Fused residual / Runge-Kutta stage kernel.
//
// One workgroup owns a TX x TY tile of cells in the (i, j) plane of a block
// and, in 3D, marches along k over KC planes.  Per plane:
//   1. primitive values of the plane with a two-cell halo in i and j are
//      staged in LDS (ghost cells included; the 3D own column comes from a
//      register queue along k);
//   2. limited slopes of eq. (flux) (slope form; one per cell and direction
//      for the symmetric limiters, a high-face/low-face pair without a
//      limiter) are computed once per cell into LDS;
//   3. the Roe flux is computed once per face of the tile (faces on the tile
//      edge are shared with the neighbour tile), the wall override of
//      Sec. 7.2 V7 applied on slip-wall faces, and stored in LDS;
//   4. every cell sums its face fluxes, divides by its volume and either
//      writes the residual or applies the stage update
//      Q^(k) = Q^(0) - alpha dt R(Q^(k-1)) (Sec. 2, M-stage Runge-Kutta) and
//      stores the new primitive state; the last stage of a step also reduces
//      Omega / lambda for the next CFL time step.
// The k direction keeps (q_k, q_k+1, q_k+2, slopes, F_k-1/2) in registers so
// every k-face flux is computed once.
#pragma once

#include "cfd_internal.h"
#include "device_math.h"

namespace cfd {

enum { MODE_RESIDUAL = 0, MODE_STAGE = 1 };

struct StageArgs {
  const BlockDev* blocks;
  const TileDev* tiles;
  const PatchDev* patches;
  int npatches;
  int tile_begin, tile_end;
  const double* qin;     // stencil state (primitive, padded, ghosts filled)
  const double* q0;      // stage-start state Q^(0) (primitive, padded)
  double* qout;          // stage output (primitive, padded)
  const double* metric;  // metric arrays
  double* Rout;          // packed residual (MODE_RESIDUAL)
  const double* dt;      // device time step
  double alpha;
  int mode;
  unsigned long long* dtmin;  // non-null: reduce Omega/lambda of the new state (bits of a positive double)
  Gas gas;
  double half_eps;       // muscl eps / 2
  double kappa;          // muscl kappa (used only without a limiter)
  double efix;
  double e2[MAXV];       // van Albada regularisation squared
};

template <int DIM>
__device__ __forceinline__ double wall_pressure(double p0, double p1) {
  return 1.5 * p0 - 0.5 * p1;
}

// true if face `face` of block b at tangential position (t1, t2) is a slip wall
__device__ __forceinline__ bool is_wall(const StageArgs& a, int b, int face, int t1, int t2) {
  for (int p = 0; p < a.npatches; ++p) {
    const PatchDev& pt = a.patches[p];
    if (pt.block == b && pt.face == face && pt.kind == PK_SLIP_WALL && t1 >= pt.lo0 && t1 < pt.lo0 + pt.len0 &&
        t2 >= pt.lo1 && t2 < pt.lo1 + pt.len1)
      return true;
  }
  return false;
}

template <int DIM>
__device__ __forceinline__ void wall_flux(double pw, const double* S, double* F) {
  F[0] = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) F[1 + d] = pw * S[d];
  F[DIM + 1] = 0.0;
}

template <int DIM, int LIM, int TX, int TY, int KC>
__global__ void __launch_bounds__(TX* TY) stage_kernel(StageArgs a) {
  constexpr int NV = DIM + 2;
  constexpr int NT = TX * TY;
  constexpr int LX = TX + 4, LY = TY + 4;
  // two slopes per cell only when Psi = 1 (the kappa-form is not symmetric there)
  constexpr int NS = LIM == LIM_NONE ? 2 : 1;
  using ML = MetricLayout<DIM>;

  __shared__ double sq[NV][LY][LX];          // plane primitives with halo
  __shared__ double ssx[NS][NV][TY][TX + 2];  // i-slopes (+, -), cells i0-1 .. i0+TX
  __shared__ double ssy[NS][NV][TY + 2][TX];  // j-slopes (+, -), cells j0-1 .. j0+TY
  __shared__ double sfx[NV][TY][TX + 1];     // i-face fluxes, faces i0 .. i0+TX
  __shared__ double sfy[NV][TY + 1][TX];     // j-face fluxes, faces j0 .. j0+TY
  __shared__ double sred[NT / 64];

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = tid / TX;
  const double he = a.half_eps;
  const double kap = a.kappa;
  double e2[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) e2[v] = a.e2[v];
  const double dt = (a.mode == MODE_STAGE) ? *a.dt : 0.0;
  const double adt = a.alpha * dt;
  double my_min = 1.0e300;

  for (int t = a.tile_begin + blockIdx.x; t < a.tile_end; t += gridDim.x) {
    const TileDev tile = a.tiles[t];
    const BlockDev B = a.blocks[tile.block];
    const int i0 = tile.i0, j0 = tile.j0;
    const int i = i0 + tx, j = j0 + ty;
    const bool own = (i < B.ni) && (j < B.nj);
    const long long vs = B.vstride;
    const double* qin = a.qin + B.origin;
    const double* met = a.metric + B.morigin;
    const int kbeg = DIM == 3 ? tile.k0 : 0;
    const int kend = DIM == 3 ? min(tile.k0 + KC, B.nk) : 1;

    // ---- k-direction register queue (3D): cells k (qc), k+1 (qn), k+2 (qnn),
    // slopes of k (scp/scm) and k+1 (snp/snm), pressure of k-1 (pprev).
    // The same three steps serve the two-step prologue and the march, so
    // every k-face flux is formed by identical code wherever it is computed.
    double qc[NV], qn[NV], qnn[NV], scp[NV], scm[NV], snp[NV], snm[NV], fzlo[NV], fzhi[NV];
    double pprev = 0.0;
    auto zload_slope = [&](int k) {  // q(k+2) and the slopes of cell k+1
#pragma unroll
      for (int v = 0; v < NV; ++v) qnn[v] = qin[v * vs + pidx(B, i, j, k + 2)];
#pragma unroll
      for (int v = 0; v < NV; ++v) cell_slopes<LIM>(qn[v] - qc[v], qnn[v] - qn[v], e2[v], kap, snp[v], snm[v]);
    };
    auto zflux = [&](int k, double* F) {  // flux through the k-face k+1 (between cells k and k+1)
      const int kf = k + 1;
      double S[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) S[c] = met[ML::S(2, c) * vs + pidx(B, i, j, kf)];
      if (kf == 0 && (B.wall_mask & (1 << 4)) && is_wall(a, tile.block, 4, i, j)) {
        wall_flux<3>(wall_pressure<3>(qn[NV - 1], qnn[NV - 1]), S, F);
      } else if (kf == B.nk && (B.wall_mask & (1 << 5)) && is_wall(a, tile.block, 5, i, j)) {
        wall_flux<3>(wall_pressure<3>(qc[NV - 1], pprev), S, F);
      } else {
        double L[NV], R[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          L[v] = qc[v] + he * scp[v];
          R[v] = qn[v] - he * snm[v];
        }
        roe_flux<3>(L, R, S, a.gas, a.efix, F);
      }
    };
    auto zrotate = [&]() {
      pprev = qc[NV - 1];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        qc[v] = qn[v];
        qn[v] = qnn[v];
        scp[v] = snp[v];
        scm[v] = snm[v];
      }
    };
    if constexpr (DIM == 3) {
      if (own) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          qc[v] = qin[v * vs + pidx(B, i, j, kbeg - 2)];
          qn[v] = qin[v * vs + pidx(B, i, j, kbeg - 1)];
        }
        zload_slope(kbeg - 2);
        zrotate();
        zload_slope(kbeg - 1);
        zflux(kbeg - 1, fzlo);
        zrotate();
      }
    }

    for (int k = kbeg; k < kend; ++k) {
      if constexpr (DIM == 3) {
        if (own) {
          zload_slope(k);
          zflux(k, fzhi);
        }
      }

      // ---- 1. stage the plane with its halo in LDS ----------------------
      if (DIM == 3 && own) {
#pragma unroll
        for (int v = 0; v < NV; ++v) sq[v][ty + 2][tx + 2] = qc[v];
      } else if (i <= B.ni + 1 && j <= B.nj + 1) {
#pragma unroll
        for (int v = 0; v < NV; ++v) sq[v][ty + 2][tx + 2] = qin[v * vs + pidx(B, i, j, k)];
      }
      // halo ring without corners: 2 rows above/below (TX wide), 2 columns left/right (TY tall)
      for (int e = tid; e < 4 * TX + 4 * TY; e += NT) {
        int lx, ly;
        if (e < 4 * TX) {
          int r = e / TX;
          lx = 2 + e % TX;
          ly = r < 2 ? r : TY + r;  // rows 0,1 and TY+2, TY+3
        } else {
          int e2i = e - 4 * TX;
          int c = e2i & 3;
          ly = 2 + (e2i >> 2);
          lx = c < 2 ? c : TX + c;  // columns 0,1 and TX+2, TX+3
        }
        const int ii = i0 - 2 + lx, jj = j0 - 2 + ly;
        if (ii <= B.ni + 1 && jj <= B.nj + 1) {
#pragma unroll
          for (int v = 0; v < NV; ++v) sq[v][ly][lx] = qin[v * vs + pidx(B, ii, jj, k)];
        }
      }
      __syncthreads();

      // ---- 2. slopes ------------------------------------------------------
      for (int e = tid; e < (TX + 2) * TY; e += NT) {
        const int c = e % (TX + 2), r = e / (TX + 2);
        const int lx = c + 1, ly = r + 2;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double sp, sm;
          cell_slopes<LIM>(sq[v][ly][lx] - sq[v][ly][lx - 1], sq[v][ly][lx + 1] - sq[v][ly][lx], e2[v], kap, sp, sm);
          ssx[0][v][r][c] = sp;
          if constexpr (NS == 2) ssx[NS - 1][v][r][c] = sm;
        }
      }
      for (int e = tid; e < TX * (TY + 2); e += NT) {
        const int c = e % TX, r = e / TX;
        const int lx = c + 2, ly = r + 1;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double sp, sm;
          cell_slopes<LIM>(sq[v][ly][lx] - sq[v][ly - 1][lx], sq[v][ly + 1][lx] - sq[v][ly][lx], e2[v], kap, sp, sm);
          ssy[0][v][r][c] = sp;
          if constexpr (NS == 2) ssy[NS - 1][v][r][c] = sm;
        }
      }
      __syncthreads();

      // ---- 3. face fluxes ---------------------------------------------------
      for (int e = tid; e < (TX + 1) * TY; e += NT) {
        const int f = e % (TX + 1), r = e / (TX + 1);
        const int fi = i0 + f, jj = j0 + r;
        if (fi <= B.ni && jj < B.nj) {
          double S[DIM], F[NV];
#pragma unroll
          for (int c = 0; c < DIM; ++c) S[c] = met[ML::S(0, c) * vs + pidx(B, fi, jj, k)];
          const int face = fi == 0 ? 0 : (fi == B.ni ? 1 : -1);
          if (face >= 0 && (B.wall_mask & (1 << face)) && is_wall(a, tile.block, face, jj, k)) {
            const double pw = face == 0 ? wall_pressure<DIM>(sq[NV - 1][r + 2][f + 2], sq[NV - 1][r + 2][f + 3])
                                        : wall_pressure<DIM>(sq[NV - 1][r + 2][f + 1], sq[NV - 1][r + 2][f]);
            wall_flux<DIM>(pw, S, F);
          } else {
            double L[NV], R[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              L[v] = sq[v][r + 2][f + 1] + he * ssx[0][v][r][f];
              R[v] = sq[v][r + 2][f + 2] - he * ssx[NS - 1][v][r][f + 1];
            }
            roe_flux<DIM>(L, R, S, a.gas, a.efix, F);
          }
#pragma unroll
          for (int v = 0; v < NV; ++v) sfx[v][r][f] = F[v];
        }
      }
      for (int e = tid; e < TX * (TY + 1); e += NT) {
        const int c = e % TX, f = e / TX;
        const int ii = i0 + c, fj = j0 + f;
        if (ii < B.ni && fj <= B.nj) {
          double S[DIM], F[NV];
#pragma unroll
          for (int cc = 0; cc < DIM; ++cc) S[cc] = met[ML::S(1, cc) * vs + pidx(B, ii, fj, k)];
          const int face = fj == 0 ? 2 : (fj == B.nj ? 3 : -1);
          if (face >= 0 && (B.wall_mask & (1 << face)) && is_wall(a, tile.block, face, ii, k)) {
            const double pw = face == 2 ? wall_pressure<DIM>(sq[NV - 1][f + 2][c + 2], sq[NV - 1][f + 3][c + 2])
                                        : wall_pressure<DIM>(sq[NV - 1][f + 1][c + 2], sq[NV - 1][f][c + 2]);
            wall_flux<DIM>(pw, S, F);
          } else {
            double L[NV], R[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              L[v] = sq[v][f + 1][c + 2] + he * ssy[0][v][f][c];
              R[v] = sq[v][f + 2][c + 2] - he * ssy[NS - 1][v][f + 1][c];
            }
            roe_flux<DIM>(L, R, S, a.gas, a.efix, F);
          }
#pragma unroll
          for (int v = 0; v < NV; ++v) sfy[v][f][c] = F[v];
        }
      }
      __syncthreads();

      // ---- 4. divergence and update ---------------------------------------
      if (own) {
        const long long ci = pidx(B, i, j, k);
        const double iv = met[ML::INVVOL * vs + ci];
        double R[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double div = (sfx[v][ty][tx + 1] - sfx[v][ty][tx]) + (sfy[v][ty + 1][tx] - sfy[v][ty][tx]);
          if constexpr (DIM == 3) div += fzhi[v] - fzlo[v];
          R[v] = div * iv;
        }
        if (a.mode == MODE_RESIDUAL) {
          const long long pc = B.packed + ((long long)k * B.nj + j) * B.ni + i;
#pragma unroll
          for (int v = 0; v < NV; ++v) a.Rout[v * B.ncell_total + pc] = R[v];
        } else {
          const double* q0 = a.q0 + B.origin;
          double w[NV], Q[NV], qnew[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) w[v] = q0[v * vs + ci];
          prim_to_cons<DIM>(w, a.gas, Q);
#pragma unroll
          for (int v = 0; v < NV; ++v) Q[v] -= adt * R[v];
          cons_to_prim<DIM>(Q, a.gas, qnew);
          double* qo = a.qout + B.origin;
#pragma unroll
          for (int v = 0; v < NV; ++v) qo[v * vs + ci] = qnew[v];
          if (a.dtmin) {
            // Omega / lambda with lambda = sum_d |u . Sbar_d| + c |Sbar_d|
            const double c = sqrt(a.gas.gamma * qnew[NV - 1] / qnew[0]);
            double lam = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
              const long long step = d == 0 ? 1 : (d == 1 ? (long long)B.pi : (long long)B.pi * B.pj);
              double un = 0.0, s2 = 0.0;
#pragma unroll
              for (int cc = 0; cc < DIM; ++cc) {
                const double sb = 0.5 * (met[ML::S(d, cc) * vs + ci] + met[ML::S(d, cc) * vs + ci + step]);
                un += qnew[1 + cc] * sb;
                s2 += sb * sb;
              }
              lam += fabs(un) + c * sqrt(s2);
            }
            my_min = fmin(my_min, 1.0 / (lam * iv));
          }
        }
      }

      if constexpr (DIM == 3) {
        if (own) {
#pragma unroll
          for (int v = 0; v < NV; ++v) fzlo[v] = fzhi[v];
          zrotate();
        }
      }
      __syncthreads();
    }
  }

  if (a.dtmin) {
    // workgroup minimum -> one atomic per workgroup
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) my_min = fmin(my_min, __shfl_xor(my_min, off));
    if ((tid & 63) == 0) sred[tid >> 6] = my_min;
    __syncthreads();
    if (tid == 0) {
      double m = sred[0];
      for (int w = 1; w < NT / 64; ++w) m = fmin(m, sred[w]);
      atomicMin(a.dtmin, (unsigned long long)__double_as_longlong(m));
    }
  }
}

}  // namespace cfd
