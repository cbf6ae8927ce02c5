// Fused residual / Runge-Kutta stage kernel.
//
// One workgroup owns a TX x TY tile of cells in the (i, j) plane of a block
// and, in 3D, marches along k over KC planes.  Per plane:
//   1. primitive values of the plane with a two-cell halo in i and j are
//      staged in LDS (ghost cells included; in 3D the tile's own cells come
//      from a register queue along k);
//   2. the limited slopes of eq. (flux) (slope form; one per cell and
//      direction for the symmetric limiters, a high-face/low-face pair without
//      a limiter) are computed once per cell into LDS;
//   3. the Roe flux is computed once per i- and j-face of the tile (faces on
//      the tile edge are shared with the neighbour tile), the wall override of
//      Sec. 7.2 V7 applied on slip-wall faces, and stored in LDS;
//   4. every cell sums its face fluxes, scales by its inverse volume and either
//      writes the residual or applies the stage update
//      Q^(k) = Q^(0) - alpha dt R(Q^(k-1)) (Sec. 2, M-stage Runge-Kutta) and
//      stores the new primitive state; the last stage of a step also reduces
//      Omega / lambda for the next CFL time step.
// Steps 2 and 3 run the i- and j-items of a plane as one flattened list with a
// single code path (per-lane addressing), so a wavefront never diverges
// between directions.  The k direction keeps (q_k, q_k+1, q_k+2, slopes,
// F_k-1/2) in registers so every k-face flux is computed once.
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
  double half_inv_efix;  // 0.5 / efix (0 when efix = 0)
  double e2[MAXV];       // van Albada regularisation squared
};

__device__ __forceinline__ double wall_pressure(double p0, double p1) { return 1.5 * p0 - 0.5 * p1; }

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
  constexpr int LX = TX + 4, LY = TY + 4, LP = LX * LY;
  // two slopes per cell only when Psi = 1 (the kappa-form is not symmetric there)
  constexpr int NS = LIM == LIM_NONE ? 2 : 1;
  constexpr int NSX = (TX + 2) * TY, NSY = TX * (TY + 2), NSL = NSX + NSY;  // slope items
  constexpr int NFX = (TX + 1) * TY, NFY = TX * (TY + 1), NFL = NFX + NFY;  // face items
  using ML = MetricLayout<DIM>;

  __shared__ double sq[NV][LP];        // plane primitives with halo, [ly][lx]
  __shared__ double sl[NS][NV][NSL];   // slopes: i-items [r][c] (c: cells i0-1..i0+TX), then j-items
  __shared__ double fl[NV][NFL];       // fluxes: i-faces [r][f] (f: faces i0..i0+TX), then j-faces [f][c]
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
  const bool q0_is_qin = a.q0 == a.qin;
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
    double qc[NV], qn[NV], qnn[NV], scp[NV], scm[NS == 2 ? NV : 1], snp[NV], snm[NS == 2 ? NV : 1];
    double fzlo[NV], fzhi[NV];
    double pprev = 0.0;
    auto zload_slope = [&](int k) {  // q(k+2) and the slopes of cell k+1
#pragma unroll
      for (int v = 0; v < NV; ++v) qnn[v] = qin[v * vs + pidx(B, i, j, k + 2)];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double sp, sm;
        cell_slopes<LIM>(qn[v] - qc[v], qnn[v] - qn[v], e2[v], kap, sp, sm);
        snp[v] = sp;
        if constexpr (NS == 2) snm[v] = sm;
      }
    };
    auto zflux = [&](int k, double* F) {  // flux through the k-face k+1 (between cells k and k+1)
      const int kf = k + 1;
      double S[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) S[c] = met[ML::S(2, c) * vs + pidx(B, i, j, kf)];
      if (kf == 0 && (B.wall_mask & (1 << 4)) && is_wall(a, tile.block, 4, i, j)) {
        wall_flux<3>(wall_pressure(qn[NV - 1], qnn[NV - 1]), S, F);
      } else if (kf == B.nk && (B.wall_mask & (1 << 5)) && is_wall(a, tile.block, 5, i, j)) {
        wall_flux<3>(wall_pressure(qc[NV - 1], pprev), S, F);
      } else {
        double L[NV], R[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          L[v] = qc[v] + he * scp[v];
          if constexpr (NS == 2)
            R[v] = qn[v] - he * snm[v];
          else
            R[v] = qn[v] - he * snp[v];
        }
        roe_flux<3>(L, R, S, a.gas, a.efix, a.half_inv_efix, F);
      }
    };
    auto zrotate = [&]() {
      pprev = qc[NV - 1];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        qc[v] = qn[v];
        qn[v] = qnn[v];
        scp[v] = snp[v];
        if constexpr (NS == 2) scm[v] = snm[v];
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
        if (own) zload_slope(k);
      }

      // ---- 1. stage the plane with its halo in LDS ----------------------
      if (DIM == 3 && own) {
#pragma unroll
        for (int v = 0; v < NV; ++v) sq[v][(ty + 2) * LX + tx + 2] = qc[v];
      } else if (i <= B.ni + 1 && j <= B.nj + 1) {
#pragma unroll
        for (int v = 0; v < NV; ++v) sq[v][(ty + 2) * LX + tx + 2] = qin[v * vs + pidx(B, i, j, k)];
      }
      // halo ring without corners: 2 rows above/below (TX wide), 2 columns left/right (TY tall)
      for (int e = tid; e < 4 * TX + 4 * TY; e += NT) {
        int lx, ly;
        if (e < 4 * TX) {
          const int r = e / TX;
          lx = 2 + e % TX;
          ly = r < 2 ? r : TY + r;  // rows 0,1 and TY+2, TY+3
        } else {
          const int e2i = e - 4 * TX;
          const int c = e2i & 3;
          ly = 2 + (e2i >> 2);
          lx = c < 2 ? c : TX + c;  // columns 0,1 and TX+2, TX+3
        }
        const int ii = i0 - 2 + lx, jj = j0 - 2 + ly;
        if (ii <= B.ni + 1 && jj <= B.nj + 1) {
#pragma unroll
          for (int v = 0; v < NV; ++v) sq[v][ly * LX + lx] = qin[v * vs + pidx(B, ii, jj, k)];
        }
      }
      __syncthreads();

      // ---- 2. slopes: i-items then j-items, one code path -----------------
      for (int e = tid; e < NSL; e += NT) {
        int p, st;
        if (e < NSX) {
          const int c = e % (TX + 2), r = e / (TX + 2);
          p = (r + 2) * LX + c + 1;
          st = 1;
        } else {
          const int e2i = e - NSX;
          const int c = e2i % TX, r = e2i / TX;
          p = (r + 1) * LX + c + 2;
          st = LX;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double sp, sm;
          cell_slopes<LIM>(sq[v][p] - sq[v][p - st], sq[v][p + st] - sq[v][p], e2[v], kap, sp, sm);
          sl[0][v][e] = sp;
          if constexpr (NS == 2) sl[NS - 1][v][e] = sm;
        }
      }
      __syncthreads();

      // ---- 3. face fluxes: i-faces then j-faces, one code path ------------
      for (int e = tid; e < NFL; e += NT) {
        int pL, st, sL, sR, fi, fj, d, face, t1;
        bool valid;
        if (e < NFX) {
          const int f = e % (TX + 1), r = e / (TX + 1);
          pL = (r + 2) * LX + f + 1;
          st = 1;
          sL = r * (TX + 2) + f;
          sR = sL + 1;
          fi = i0 + f;
          fj = j0 + r;
          d = 0;
          face = fi == 0 ? 0 : (fi == B.ni ? 1 : -1);
          t1 = fj;
          valid = fi <= B.ni && fj < B.nj;
        } else {
          const int e2i = e - NFX;
          const int c = e2i % TX, f = e2i / TX;
          pL = (f + 1) * LX + c + 2;
          st = LX;
          sL = NSX + f * TX + c;
          sR = sL + TX;
          fi = i0 + c;
          fj = j0 + f;
          d = 1;
          face = fj == 0 ? 2 : (fj == B.nj ? 3 : -1);
          t1 = fi;
          valid = fi < B.ni && fj <= B.nj;
        }
        if (valid) {
          double S[DIM], F[NV];
          const long long fidx = pidx(B, fi, fj, k);
#pragma unroll
          for (int c = 0; c < DIM; ++c) S[c] = met[ML::S(d, c) * vs + fidx];
          if (face >= 0 && (B.wall_mask & (1 << face)) && is_wall(a, tile.block, face, t1, k)) {
            // p0 = cell next to the wall, p1 = the one after it
            const int pin = (face & 1) ? pL : pL + st;
            const int dir = (face & 1) ? -st : st;
            wall_flux<DIM>(wall_pressure(sq[NV - 1][pin], sq[NV - 1][pin + dir]), S, F);
          } else {
            double L[NV], R[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              L[v] = sq[v][pL] + he * sl[0][v][sL];
              R[v] = sq[v][pL + st] - he * sl[NS - 1][v][sR];
            }
            roe_flux<DIM>(L, R, S, a.gas, a.efix, a.half_inv_efix, F);
          }
#pragma unroll
          for (int v = 0; v < NV; ++v) fl[v][e] = F[v];
        }
      }
      if constexpr (DIM == 3) {
        if (own) zflux(k, fzhi);
      }
      __syncthreads();

      // ---- 4. divergence and update ---------------------------------------
      if (own) {
        const long long ci = pidx(B, i, j, k);
        const double iv = met[ML::INVVOL * vs + ci];
        const int ex = ty * (TX + 1) + tx;  // i-face on this cell's low side
        const int ey = NFX + ty * TX + tx;  // j-face on this cell's low side
        double R[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double div = (fl[v][ex + 1] - fl[v][ex]) + (fl[v][ey + TX] - fl[v][ey]);
          if constexpr (DIM == 3) div += fzhi[v] - fzlo[v];
          R[v] = div * iv;
        }
        if (a.mode == MODE_RESIDUAL) {
          const long long pc = B.packed + ((long long)k * B.nj + j) * B.ni + i;
#pragma unroll
          for (int v = 0; v < NV; ++v) a.Rout[v * B.ncell_total + pc] = R[v];
        } else {
          double w[NV], Q[NV], qnew[NV];
          if (q0_is_qin) {
#pragma unroll
            for (int v = 0; v < NV; ++v) w[v] = sq[v][(ty + 2) * LX + tx + 2];
          } else {
            const double* q0 = a.q0 + B.origin;
#pragma unroll
            for (int v = 0; v < NV; ++v) w[v] = q0[v * vs + ci];
          }
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
