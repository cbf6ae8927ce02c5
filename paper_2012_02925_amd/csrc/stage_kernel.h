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
//   3. the face flux (Roe, or a flux-vector splitting) is computed once per
//      i- and j-face of the tile (faces on the tile edge are shared with the
//      neighbour tile), the override of Sec. 7.2 V7 applied on slip-wall
//      faces (wall pressure only) and farfield faces (exact flux of the
//      boundary state in the ghost cell), and stored in LDS;
//   4. every cell sums its face fluxes, scales by its inverse volume and either
//      writes the residual or applies the stage update
//      Q^(k) = Q^(0) - alpha dt R(Q^(k-1)) (Sec. 2, M-stage Runge-Kutta) and
//      stores the new primitive state; the last stage of a step also reduces
//      Omega / lambda for the next CFL time step.
// Every thread computes the slopes of its own cell and the fluxes through its
// own cell's low faces; the halo cells' slopes and the faces on the tile's
// high edges are a short extra round.  The k direction keeps q_k, q_k+1, the
// slope of k and F_k-1/2 in registers so every k-face flux is computed once.
// Global latency is hidden by prefetching: the next plane's halo item and
// q_k+3 are loaded while the current plane computes, and the own cell's
// metrics and stage-start state are loaded before the plane's first barrier.
// Those loads are issued by every lane, without a branch, from addresses kept
// in bounds (lanes without a cell read a cell of the block): where a load is
// issued under a condition, the compiler's wait counting cannot tell at the
// join how many loads are still in flight and waits for all of them, so a
// prefetch issued just before would be waited for at once.
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
                              // into DT_SLOTS slots
  double* dtloc;         // non-null: local time steps, packed per cell; read for the update and, with
                         // dtmin, overwritten by cfl * Omega/lambda of the new state
  double cfl;
  Gas gas;
  double half_eps;       // muscl eps / 2
  double kappa;          // muscl kappa (used only without a limiter)
  double efix;
  double half_inv_efix;  // 0.5 / efix (0 when efix = 0)
  double e2[MAXV];       // van Albada regularisation squared
  const double* phi;     // frozen limiter factors (LIM_FROZEN): padded arrays d * nvar + v
  const double* rv;      // viscous residual (momentum.., energy), packed, subtracted from R; or null
  double visc_cv;        // viscous time-step coefficient 4 max(4/3, gamma/Pr) mu (0: inviscid)
  int wrap;              // read periodic neighbours through the wrap of the block (BlockDev::wrap)
};

__device__ __forceinline__ double wall_pressure(double p0, double p1) { return 1.5 * p0 - 0.5 * p1; }

// true if face `face` of block b at tangential position (t1, t2) belongs to a
// patch whose kind is in the bit set `kinds` (walls and farfield faces
// overwrite the flux)
__device__ __forceinline__ bool patch_at(const StageArgs& a, int kinds, int b, int face, int t1, int t2) {
  for (int p = 0; p < a.npatches; ++p) {
    const PatchDev& pt = a.patches[p];
    if (pt.block == b && pt.face == face && ((kinds >> pt.kind) & 1) && t1 >= pt.lo0 && t1 < pt.lo0 + pt.len0 &&
        t2 >= pt.lo1 && t2 < pt.lo1 + pt.len1)
      return true;
  }
  return false;
}
__device__ __forceinline__ bool is_wall(const StageArgs& a, const BlockDev& B, int b, int face, int t1, int t2) {
  return face >= 0 && (B.wall_mask & (1 << face)) &&
         patch_at(a, (1 << PK_SLIP_WALL) | (1 << PK_NOSLIP_WALL), b, face, t1, t2);
}
__device__ __forceinline__ bool is_farfield(const StageArgs& a, const BlockDev& B, int b, int face, int t1, int t2) {
  return face >= 0 && (B.wall_mask & (FARFIELD_MASK_SHIFT << face)) && patch_at(a, 1 << PK_FARFIELD, b, face, t1, t2);
}

// Load through a uniform array base and a per-lane 32-bit byte offset (the
// host guarantees one padded array of a block stays below 4 GiB), so lanes
// keep one 32-bit offset instead of a 64-bit address per array.
__device__ __forceinline__ double ld_at(const double* base, unsigned boff) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + boff);
}
__device__ __forceinline__ void st_at(double* base, unsigned boff, double x) {
  *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + boff) = x;
}
// Non-temporal forms for data each launch touches once (the own cell's
// metrics and stage-start state, the stage output): they stream through L2
// with low retention, so the state values that neighbouring tiles re-read as
// halo stay cached longer (HBM traffic 1.20x -> 1.11x of the algorithmic
// bytes on the 256^3 box).
__device__ __forceinline__ double ld_nt(const double* base, unsigned boff) {
  return __builtin_nontemporal_load(reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) + boff));
}
__device__ __forceinline__ void st_nt(double* base, unsigned boff, double x) {
  __builtin_nontemporal_store(x, reinterpret_cast<double*>(reinterpret_cast<char*>(base) + boff));
}

template <int DIM>
__device__ __forceinline__ void wall_flux(double pw, const double* S, double* F) {
  F[0] = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) F[1 + d] = pw * S[d];
  F[DIM + 1] = 0.0;
}

// Farfield faces carry the exact flux of the boundary state q_b that the
// ghost cell holds.  Both face states are set to q_b and the scheme's flux is
// evaluated on them: every flux here is consistent, F(q, q) = F(q) (the Roe
// dissipation multiplies state jumps, the split parts sum to the flux), so
// this is the exact flux up to rounding and shares the flux code.
template <int NV>
__device__ __forceinline__ void farfield_states(const double* qb, double* L, double* R) {
#pragma unroll
  for (int v = 0; v < NV; ++v) L[v] = R[v] = qb[v];
}

// LDS bytes of one stage-kernel workgroup (must match the arrays below)
template <int DIM, int LIM, int TX, int TY>
constexpr int stage_lds_bytes() {
  constexpr int NV = DIM + 2, NS = LIM == LIM_NONE ? 2 : 1;
  return 8 * (NV * (TX + 4) * (TY + 4) + NS * NV * (TX + 2) * TY + NS * NV * TX * (TY + 2) + NV * (TX + 1) * TY +
              NV * TX * (TY + 1) + (DIM == 3 ? NV * TX * TY : 1) + TX * TY / 64);
}
// waves per SIMD that the LDS footprint allows (160 KiB per CU, 4 SIMDs); the
// register allocation is asked to fit the same number
template <int DIM, int LIM, int TX, int TY>
constexpr int stage_waves() {
  constexpr int wg = (160 * 1024) / stage_lds_bytes<DIM, LIM, TX, TY>();
  constexpr int w = wg * (TX * TY / 64) / 4;
  return w < 1 ? 1 : (w > 8 ? 8 : w);
}

// FF: the launch has farfield faces.  Kernels without them keep the farfield
// test out of the face loops, whose register budget is tight in 3D.
// DT: the launch reduces Omega / lambda for the next time step (a.dtmin set,
// the last stage of a step).  The other stages run an instantiation without
// that epilogue, so its loads and registers do not weigh on them.
template <int DIM, int LIM, int TX, int TY, int KC, int FLUX, bool FF, bool DT>
__global__ void __launch_bounds__(TX* TY) __attribute__((amdgpu_waves_per_eu(stage_waves<DIM, LIM, TX, TY>())))
stage_kernel(StageArgs a) {
  constexpr int NV = DIM + 2;
  constexpr int NT = TX * TY;
  constexpr int LX = TX + 4, LY = TY + 4, LP = LX * LY;
  // two slopes per cell only when Psi = 1 (the kappa-form is not symmetric there)
  constexpr int NS = LIM == LIM_NONE ? 2 : 1;
  constexpr int SXW = TX + 2;         // i-slope rows: cells i0-1 .. i0+TX
  constexpr int NSX = SXW * TY;
  constexpr int NSY = TX * (TY + 2);  // j-slope rows j0-1 .. j0+TY
  constexpr int FXW = TX + 1;         // i-face rows: faces i0 .. i0+TX
  constexpr int NFX = FXW * TY;
  constexpr int NFY = TX * (TY + 1);  // j-face rows j0 .. j0+TY
  constexpr int NHALO = 4 * TX + 4 * TY;
  constexpr int NXS = 2 * TY + 2 * TX;  // slopes of the halo cells
  constexpr int NXF = TY + TX;          // faces on the tile's high edges
  using ML = MetricLayout<DIM>;
  constexpr int NH = (NHALO + NT - 1) / NT;  // halo items per thread
  constexpr int NWAVE = NT / 64;
  static_assert(NXS <= NT && NXF <= NT, "tile too flat for one halo slope per thread");
  static_assert(NT % 64 == 0, "whole wavefronts per workgroup");

  __shared__ double sq[NV][LP];        // plane primitives with halo, [ly][lx]
  __shared__ double slx[NS][NV][NSX];  // i-slopes (+, -)
  __shared__ double sly[NS][NV][NSY];  // j-slopes (+, -)
  __shared__ double flx[NV][NFX];      // i-face fluxes
  __shared__ double fly[NV][NFY];      // j-face fluxes
  __shared__ double fzs[DIM == 3 ? NV : 1][DIM == 3 ? NT : 1];  // lower k-face flux of the own cell
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
  const bool update = a.mode == MODE_STAGE;
  double my_min = 1.0e300;
  const int own_lp = (ty + 2) * LX + tx + 2;

  for (int t = a.tile_begin + blockIdx.x; t < a.tile_end; t += gridDim.x) {
    const TileDev tile = a.tiles[t];
    const BlockDev B = a.blocks[tile.block];
    const int i0 = tile.i0, j0 = tile.j0;
    const int i = i0 + tx, j = j0 + ty;
    const bool own = (i < B.ni) && (j < B.nj);
    const bool own_in_pad = (i <= B.ni + 1) && (j <= B.nj + 1);
    // the low faces of the own cell exist up to the block's high faces
    const bool fx_ok = (i <= B.ni) && (j < B.nj);
    const bool fy_ok = (i < B.ni) && (j <= B.nj);
    const long long vs = B.vstride;
    const long long plane = (long long)B.pi * B.pj;
    // array bases (lowest ghost cell of array 0) and byte offsets from them
    const long long K = (DIM == 3 ? 2LL * B.pj + 2 : 2LL) * B.pi + 2;
    const double* qin = a.qin + (B.origin - K);
    const double* met = a.metric + (B.morigin - K);
    const double* phib = LIM == LIM_FROZEN ? a.phi + (B.lorigin - K) : nullptr;
    const unsigned p8 = (unsigned)plane * 8u;
    const int kbeg = DIM == 3 ? tile.k0 : 0;
    const int kend = DIM == 3 ? min(tile.k0 + KC, B.nk) : 1;
    // own column, plane 0; lanes beyond the padded block take the block's
    // first column so every load below has an in-bounds address and can be
    // issued without a branch (conditionally issued loads make the compiler
    // wait for all outstanding loads, prefetches included, where the paths
    // join)
    const long long oc = (own_in_pad ? pidx(B, i, j, 0) : 0) + K;
    // (metrics, stage-start state and output of the lane's cell, plane k)
    auto zoff = [&](int k) { return (unsigned)((oc + (long long)k * plane) * 8); };
    // Along an axis that the block connects to itself end to end, the stencil
    // reads the cells that the ghost cells copy (the same values), so the
    // ghost fill between stages can leave those connections out.  Only state
    // values are read through the wrap: a lane on a ghost cell of the high
    // side still takes the area vector of its own low face, the block's
    // boundary face, from its unwrapped position.
    const int wrap = a.wrap ? B.wrap : 0;
    auto wrapc = [](int x, int n, bool on) { return on ? (x < 0 ? x + n : (x >= n ? x - n : x)) : x; };
    const long long ocq =
        (own_in_pad ? pidx(B, wrapc(i, B.ni, wrap & 1), wrapc(j, B.nj, wrap & 2), 0) : 0) + K;
    // the lane's state in plane k (the k-queue's ghost planes k < 0, k >= nk through the wrap)
    auto zq = [&](int k) {
      return (unsigned)((ocq + (long long)wrapc(k, B.nk, DIM == 3 && (wrap & 4)) * plane) * 8);
    };

    // this thread's halo-ring items (the same for every plane of the tile)
    int hpos[NH];
    unsigned hoff[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int e0 = tid + h * NT;
      hpos[h] = -1;
      hoff[h] = 0;
      if (e0 < NHALO) {
        int lx, ly;
        if (e0 < 4 * TX) {
          const int r = e0 / TX;
          lx = 2 + e0 % TX;
          ly = r < 2 ? r : TY + r;  // rows 0,1 and TY+2, TY+3
        } else {
          const int e = e0 - 4 * TX;
          const int c = e & 3;
          ly = 2 + (e >> 2);
          lx = c < 2 ? c : TX + c;  // columns 0,1 and TX+2, TX+3
        }
        const int ii = i0 - 2 + lx, jj = j0 - 2 + ly;
        if (ii <= B.ni + 1 && jj <= B.nj + 1) {
          hpos[h] = ly * LX + lx;
          hoff[h] = (unsigned)((pidx(B, wrapc(ii, B.ni, wrap & 1), wrapc(jj, B.nj, wrap & 2), 0) + K) * 8);
        }
      }
    }
    // Lanes of rank rs < NXS take a halo cell's slope, lanes of rank re < NXF
    // a face on the tile's high edges.  In 2D (one plane per tile) the ranks
    // rotate over the waves from tile to tile, so this extra work does not
    // always fall on the same SIMD of a compute unit; in 3D they are tid.
    const int rot = DIM == 2 ? t % NWAVE : 0;
    const int rs = DIM == 2 ? (tid + NT - 64 * ((rot + 1) % NWAVE)) % NT : tid;
    const int re = DIM == 2 ? (tid + NT - 64 * rot) % NT : tid;
    // this lane's face on the tile's high edges: i-face i0+TX of row re, then
    // j-face j0+TY of column re-TY; plane-0 offset of its area vector (an
    // in-bounds cell where the face lies outside the block)
    int edge_d = 0;
    unsigned edge_off = 0;
    if (re < NXF) {
      const int fi = re < TY ? i0 + TX : i0 + re - TY;
      const int fj = re < TY ? j0 + re : j0 + TY;
      edge_d = re < TY ? 0 : 1;
      if (fi <= B.ni + 1 && fj <= B.nj + 1) edge_off = (unsigned)((pidx(B, fi, fj, 0) + K) * 8);
    }
    double pre_h[NH][NV];  // prefetched halo values of the next plane
    // unused items load the block's first cell (hoff = 0)
    auto fetch_halo = [&](int k) {
#pragma unroll
      for (int h = 0; h < NH; ++h) {
#pragma unroll
        for (int v = 0; v < NV; ++v) pre_h[h][v] = ld_at(qin + v * vs, hoff[h] + k * p8);
      }
    };

    // ---- k-direction register queue (3D): cells k (qc), k+1 (qn), slopes of
    // k (scp/scm) and the prefetched q(k+2) (qnx); the lower k-face flux of
    // the own cell waits in LDS (only its own thread touches that slot).
    // Inside a plane q(k) is read back from LDS, so qc is dead there.
    double qc[NV], qn[NV], qnx[NV], scp[NV], scm[NS == 2 ? NV : 1], fzd[NV];
    // (DT, 3D) area vector of the own cell's low k-face: the previous plane's Sz
    double szlo[DT && DIM == 3 ? 3 : 1];
    double pprev = 0.0;
    // slopes of cell k+1 from q(k), q(k+1), q(k+2); flux of face k+1; shift the queue
    auto zstep = [&](int k, const double* qcur, const double* qnn, const double* Sz, double* F) {
      double snp[NV], snm[NS == 2 ? NV : 1];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double sp, sm;
        if constexpr (LIM == LIM_FROZEN)
          sp = frozen_slope(ld_at(phib + (2 * NV + v) * vs, zoff(k + 1)), qn[v] - qcur[v], qnn[v] - qn[v]);
        else
          cell_slopes<LIM>(qn[v] - qcur[v], qnn[v] - qn[v], e2[v], kap, sp, sm);
        snp[v] = sp;
        if constexpr (NS == 2) snm[v] = sm;
      }
      if (F) {
        const int kf = k + 1;
        if (kf == 0 && is_wall(a, B, tile.block, 4, i, j)) {
          wall_flux<3>(wall_pressure(qn[NV - 1], qnn[NV - 1]), Sz, F);
        } else if (kf == B.nk && is_wall(a, B, tile.block, 5, i, j)) {
          wall_flux<3>(wall_pressure(qcur[NV - 1], pprev), Sz, F);
        } else {
          double L[NV], R[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            L[v] = qcur[v] + he * scp[v];
            if constexpr (NS == 2)
              R[v] = qn[v] - he * snm[v];
            else
              R[v] = qn[v] - he * snp[v];
          }
          if (FF && kf == 0 && is_farfield(a, B, tile.block, 4, i, j)) farfield_states<NV>(qcur, L, R);
          if (FF && kf == B.nk && is_farfield(a, B, tile.block, 5, i, j)) farfield_states<NV>(qn, L, R);
          face_flux<3, FLUX>(L, R, Sz, a.gas, a.efix, a.half_inv_efix, F);
        }
      }
      pprev = qcur[NV - 1];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        qc[v] = qn[v];
        qn[v] = qnn[v];
        scp[v] = snp[v];
        if constexpr (NS == 2) scm[v] = snm[v];
      }
    };
    if constexpr (DIM == 3) {
      {  // every lane (lanes without a cell work on an in-bounds column; results unused)
        double q2[NV], Sz[3];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          qc[v] = ld_at(qin + v * vs, zq(kbeg - 2));
          qn[v] = ld_at(qin + v * vs, zq(kbeg - 1));
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) q2[v] = ld_at(qin + v * vs, zq(kbeg));
        zstep(kbeg - 2, qc, q2, nullptr, nullptr);
#pragma unroll
        for (int v = 0; v < NV; ++v) q2[v] = ld_at(qin + v * vs, zq(kbeg + 1));
#pragma unroll
        for (int c = 0; c < 3; ++c) Sz[c] = ld_at(met + ML::S(2, c) * vs, zoff(kbeg));
        if constexpr (DT) {
#pragma unroll
          for (int c = 0; c < 3; ++c) szlo[c] = Sz[c];
        }
        zstep(kbeg - 1, qc, q2, Sz, fzd);
#pragma unroll
        for (int v = 0; v < NV; ++v) fzs[v][tid] = fzd[v];
        // queue now: qc = q(kbeg), qn = q(kbeg+1), scp = slope(kbeg)
#pragma unroll
        for (int v = 0; v < NV; ++v) qnx[v] = ld_at(qin + v * vs, zq(kbeg + 2));
      }
    }
    fetch_halo(kbeg);

    for (int k = kbeg; k < kend; ++k) {
      const unsigned ok = zoff(k);  // own cell in plane k (byte offset)
      // own-cell metrics and stage-start state of this plane, consumed after
      // the slope phase
      double Sx[DIM], Sy[DIM], Sz[DIM], Se[DIM];
#pragma unroll
      for (int c = 0; c < DIM; ++c) {
        // (the last stage's time-step epilogue reads the neighbours' low
        // faces again, so there they stay cacheable)
        Sx[c] = DT ? ld_at(met + ML::S(0, c) * vs, ok) : ld_nt(met + ML::S(0, c) * vs, ok);
        Sy[c] = DT ? ld_at(met + ML::S(1, c) * vs, ok) : ld_nt(met + ML::S(1, c) * vs, ok);
        if (DIM == 3) Sz[c] = ld_nt(met + ML::S(2, c) * vs, ok + p8);
      }
      // area vector of this lane's face on the tile's high edge (issued
      // before the halo prefetch, so waiting for it never waits for that)
      if (re < NXF) {
#pragma unroll
        for (int c = 0; c < DIM; ++c) Se[c] = ld_at(met + ML::S(edge_d, c) * vs, edge_off + k * p8);
      }

      // ---- 1. stage the plane with its halo in LDS ----------------------
      if (DIM == 3 && own) {
#pragma unroll
        for (int v = 0; v < NV; ++v) sq[v][own_lp] = qc[v];
      } else if (own_in_pad) {
        const unsigned okq = zq(k);
#pragma unroll
        for (int v = 0; v < NV; ++v) sq[v][own_lp] = ld_at(qin + v * vs, okq);
      }
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        if (hpos[h] >= 0) {
#pragma unroll
          for (int v = 0; v < NV; ++v) sq[v][hpos[h]] = pre_h[h][v];
        }
      }
      __syncthreads();
      // prefetch the next plane's halo while this plane computes
      if (DIM == 3) fetch_halo(k + 1 < kend ? k + 1 : k);

      // ---- 2. slopes: own cell (i and j), then the halo cells ------------
      {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double sp, sm;
          if constexpr (LIM == LIM_FROZEN) {
            // cells beyond the padded block compute slopes nobody reads
            const double fx = ld_at(phib + v * vs, ok);
            const double fy = ld_at(phib + (NV + v) * vs, ok);
            slx[0][v][ty * SXW + tx + 1] =
                frozen_slope(fx, sq[v][own_lp] - sq[v][own_lp - 1], sq[v][own_lp + 1] - sq[v][own_lp]);
            sly[0][v][(ty + 1) * TX + tx] =
                frozen_slope(fy, sq[v][own_lp] - sq[v][own_lp - LX], sq[v][own_lp + LX] - sq[v][own_lp]);
            continue;
          }
          cell_slopes<LIM>(sq[v][own_lp] - sq[v][own_lp - 1], sq[v][own_lp + 1] - sq[v][own_lp], e2[v], kap, sp,
                           sm);
          slx[0][v][ty * SXW + tx + 1] = sp;
          if constexpr (NS == 2) slx[NS - 1][v][ty * SXW + tx + 1] = sm;
          cell_slopes<LIM>(sq[v][own_lp] - sq[v][own_lp - LX], sq[v][own_lp + LX] - sq[v][own_lp], e2[v], kap, sp,
                           sm);
          sly[0][v][(ty + 1) * TX + tx] = sp;
          if constexpr (NS == 2) sly[NS - 1][v][(ty + 1) * TX + tx] = sm;
        }
      }
      if (rs < NXS) {
        int p, st, dst, hi, hj;  // LDS cell, stride, slope slot, block cell
        bool isx;
        if (rs < 2 * TY) {  // i-slopes of cells i0-1 and i0+TX
          const int r = rs >> 1, side = rs & 1;
          const int c = side ? TX + 1 : 0;
          p = (r + 2) * LX + c + 1;
          st = 1;
          dst = r * SXW + c;
          isx = true;
          hi = i0 - 1 + c;
          hj = j0 + r;
        } else {  // j-slopes of rows j0-1 and j0+TY
          const int e = rs - 2 * TY;
          const int c = e % TX, side = e / TX;
          const int r = side ? TY + 1 : 0;
          p = (r + 1) * LX + c + 2;
          st = LX;
          dst = r * TX + c;
          isx = false;
          hi = i0 + c;
          hj = j0 - 1 + r;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double sp, sm;
          if constexpr (LIM == LIM_FROZEN) {
            const bool in_pad = hi <= B.ni + 1 && hj <= B.nj + 1;
            const double f =
                in_pad ? ld_at(phib + ((isx ? 0 : NV) + v) * vs, (unsigned)((pidx(B, hi, hj, k) + K) * 8)) : 0.0;
            sp = frozen_slope(f, sq[v][p] - sq[v][p - st], sq[v][p + st] - sq[v][p]);
          } else {
            cell_slopes<LIM>(sq[v][p] - sq[v][p - st], sq[v][p + st] - sq[v][p], e2[v], kap, sp, sm);
          }
          if (isx) {
            slx[0][v][dst] = sp;
            if constexpr (NS == 2) slx[NS - 1][v][dst] = sm;
          } else {
            sly[0][v][dst] = sp;
            if constexpr (NS == 2) sly[NS - 1][v][dst] = sm;
          }
        }
      }
      __syncthreads();

      // ---- 3. face fluxes ---------------------------------------------------
      // low i-face and low j-face of the own cell (in a ragged tile also the
      // block's high faces, which are the low faces of its first ghost cells)
      double F[NV];
      if (fx_ok) {
        const int face = i == 0 ? 0 : (i == B.ni ? 1 : -1);
        if (is_wall(a, B, tile.block, face, j, k)) {
          const double pw = face == 0 ? wall_pressure(sq[NV - 1][own_lp], sq[NV - 1][own_lp + 1])
                                      : wall_pressure(sq[NV - 1][own_lp - 1], sq[NV - 1][own_lp - 2]);
          wall_flux<DIM>(pw, Sx, F);
        } else {
          double L[NV], R[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            L[v] = sq[v][own_lp - 1] + he * slx[0][v][ty * SXW + tx];
            R[v] = sq[v][own_lp] - he * slx[NS - 1][v][ty * SXW + tx + 1];
          }
          if (FF && is_farfield(a, B, tile.block, face, j, k)) {
            const int gp = face == 0 ? own_lp - 1 : own_lp;
#pragma unroll
            for (int v = 0; v < NV; ++v) L[v] = R[v] = sq[v][gp];
          }
          face_flux<DIM, FLUX>(L, R, Sx, a.gas, a.efix, a.half_inv_efix, F);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) flx[v][ty * FXW + tx] = F[v];
      }
      if (fy_ok) {
        const int face = j == 0 ? 2 : (j == B.nj ? 3 : -1);
        if (is_wall(a, B, tile.block, face, i, k)) {
          const double pw = face == 2 ? wall_pressure(sq[NV - 1][own_lp], sq[NV - 1][own_lp + LX])
                                      : wall_pressure(sq[NV - 1][own_lp - LX], sq[NV - 1][own_lp - 2 * LX]);
          wall_flux<DIM>(pw, Sy, F);
        } else {
          double L[NV], R[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            L[v] = sq[v][own_lp - LX] + he * sly[0][v][ty * TX + tx];
            R[v] = sq[v][own_lp] - he * sly[NS - 1][v][(ty + 1) * TX + tx];
          }
          if (FF && is_farfield(a, B, tile.block, face, i, k)) {
            const int gp = face == 2 ? own_lp - LX : own_lp;
#pragma unroll
            for (int v = 0; v < NV; ++v) L[v] = R[v] = sq[v][gp];
          }
          face_flux<DIM, FLUX>(L, R, Sy, a.gas, a.efix, a.half_inv_efix, F);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) fly[v][ty * TX + tx] = F[v];
      }
      // faces on the tile's high edges: i-face i0+TX of each row, j-face j0+TY of each column
      if (re < NXF) {
        int pL, st, sL, sR, fi, fj, dst;
        bool isx;
        if (re < TY) {
          const int r = re;
          pL = (r + 2) * LX + TX + 1;
          st = 1;
          sL = r * SXW + TX;
          sR = sL + 1;
          fi = i0 + TX;
          fj = j0 + r;
          dst = r * FXW + TX;
          isx = true;
        } else {
          const int c = re - TY;
          pL = (TY + 1) * LX + c + 2;
          st = LX;
          sL = TY * TX + c;
          sR = sL + TX;
          fi = i0 + c;
          fj = j0 + TY;
          dst = TY * TX + c;
          isx = false;
        }
        const bool valid = isx ? (fi <= B.ni && fj < B.nj) : (fi < B.ni && fj <= B.nj);
        if (valid) {
          const double* S = Se;
          double F[NV];
          const int face = isx ? (fi == B.ni ? 1 : -1) : (fj == B.nj ? 3 : -1);
          if (is_wall(a, B, tile.block, face, isx ? fj : fi, k)) {
            wall_flux<DIM>(wall_pressure(sq[NV - 1][pL], sq[NV - 1][pL - st]), S, F);
          } else {
            double L[NV], R[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              L[v] = sq[v][pL] + he * (isx ? slx[0][v][sL] : sly[0][v][sL]);
              R[v] = sq[v][pL + st] - he * (isx ? slx[NS - 1][v][sR] : sly[NS - 1][v][sR]);
            }
            if (FF && is_farfield(a, B, tile.block, face, isx ? fj : fi, k)) {
#pragma unroll
              for (int v = 0; v < NV; ++v) L[v] = R[v] = sq[v][pL + st];
            }
            face_flux<DIM, FLUX>(L, R, S, a.gas, a.efix, a.half_inv_efix, F);
          }
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            if (isx)
              flx[v][dst] = F[v];
            else
              fly[v][dst] = F[v];
          }
        }
      }
      // inverse volume, stage-start state and (local stepping) the cell's time
      // step, consumed after the next barrier
      // (every lane loads; lanes without a cell read an in-bounds cell)
      double w0[NV], adtc = adt;
      const long long pcell = B.packed + (own ? ((long long)k * B.nj + j) * B.ni + i : 0);
      const double iv = ld_nt(met + ML::INVVOL * vs, ok);
      // (DT) the cell's high i- and j-face area vectors, consumed after the next barrier
      double shi[DT ? 2 : 1][DIM];
      if constexpr (DT) {
#pragma unroll
        for (int cc = 0; cc < DIM; ++cc) {
          shi[0][cc] = ld_at(met + ML::S(0, cc) * vs, ok + 8u);
          shi[1][cc] = ld_at(met + ML::S(1, cc) * vs, ok + 8u * B.pi);
        }
      }
      if (update && a.dtloc) adtc = a.alpha * a.dtloc[pcell];
      if (update && !q0_is_qin) {
        const double* q0 = a.q0 + (B.origin - K);
#pragma unroll
        for (int v = 0; v < NV; ++v) w0[v] = ld_nt(q0 + v * vs, ok);
      }
      double rvc[NV - 1];  // viscous residual of the cell (Navier-Stokes)
      if (a.rv) {
#pragma unroll
        for (int v = 1; v < NV; ++v) rvc[v - 1] = a.rv[(v - 1) * B.ncell_total + pcell];
      }
      // k-face k+1 of the own column (queue: q(k) in LDS, q(k+1), q(k+2)), then
      // the k part of the divergence; prefetch q(k+3) for the next plane (the
      // current plane again after the tile's last plane).  Lanes without a
      // cell compute on their in-bounds column and their results are unused.
      if constexpr (DIM == 3) {
        double qcur[NV], fz[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) qcur[v] = sq[v][own_lp];
        zstep(k, qcur, qnx, Sz, fz);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          fzd[v] = fz[v] - fzs[v][tid];
          fzs[v][tid] = fz[v];
        }
        const unsigned o3 = zq(k + 1 < kend ? k + 3 : k);
#pragma unroll
        for (int v = 0; v < NV; ++v) qnx[v] = ld_at(qin + v * vs, o3);
      }
      __syncthreads();

      // ---- 4. divergence and update ---------------------------------------
      // (DT) mean area vectors Sbar_d of the cell, ahead of the divergence:
      // the own low i- and j-faces (Sx, Sy) and both k-faces (szlo, Sz) are
      // still in registers, the high i- and j-faces were loaded before the
      // barrier above
      double sbar[DT ? DIM : 1][DIM];
      if constexpr (DT) {
#pragma unroll
        for (int cc = 0; cc < DIM; ++cc) {
          sbar[0][cc] = 0.5 * (Sx[cc] + shi[0][cc]);
          sbar[1][cc] = 0.5 * (Sy[cc] + shi[1][cc]);
          if constexpr (DIM == 3) {
            sbar[2][cc] = 0.5 * (szlo[cc] + Sz[cc]);
            szlo[cc] = Sz[cc];
          }
        }
      }
      if (own) {
        const int ex = ty * FXW + tx;
        const int ey = ty * TX + tx;
        double R[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          double div = (flx[v][ex + 1] - flx[v][ex]) + (fly[v][ey + TX] - fly[v][ey]);
          if constexpr (DIM == 3) div += fzd[v];
          R[v] = div * iv;
        }
        if (a.rv) {
#pragma unroll
          for (int v = 1; v < NV; ++v) R[v] -= rvc[v - 1];
        }
        if (!update) {
#pragma unroll
          for (int v = 0; v < NV; ++v) a.Rout[v * B.ncell_total + pcell] = R[v];
        } else {
          double Q[NV], qnew[NV];
          if (q0_is_qin) {
#pragma unroll
            for (int v = 0; v < NV; ++v) w0[v] = sq[v][own_lp];
          }
          prim_to_cons<DIM>(w0, a.gas, Q);
#pragma unroll
          for (int v = 0; v < NV; ++v) Q[v] -= adtc * R[v];
          cons_to_prim<DIM>(Q, a.gas, qnew);
          double* qo = a.qout + (B.origin - K);
#pragma unroll
          for (int v = 0; v < NV; ++v) st_nt(qo + v * vs, ok, qnew[v]);
          if constexpr (DT) {
            // Omega / lambda with lambda = sum_d |u . Sbar_d| + c |Sbar_d|
            // (reciprocal and square roots from the hardware estimates with a
            // Newton step: the step needs no correct rounding)
            const double c2 = a.gas.gamma * qnew[NV - 1] * rcp(qnew[0]);
            const double c = c2 * rsq(c2);
            double lam = 0.0, s2sum = 0.0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
              double un = 0.0, s2 = 0.0;
#pragma unroll
              for (int cc = 0; cc < DIM; ++cc) {
                const double sb = sbar[d][cc];
                un += qnew[1 + cc] * sb;
                s2 += sb * sb;
              }
              lam += fabs(un) + c * (s2 > 0.0 ? s2 * rsq(s2) : 0.0);
              s2sum += s2;
            }
            if (a.visc_cv > 0.0) lam += a.visc_cv / qnew[0] * s2sum * iv;
            const double om = rcp(lam * iv);
            my_min = fmin(my_min, om);
            if (a.dtloc) a.dtloc[pcell] = a.cfl * om;
          }
        }
      }
      // No barrier here: the next plane's staging writes sq, whose last
      // reads by other threads (face states) precede the barrier above, and
      // flx/fly, read just now, are written again only after two barriers.
    }
  }

  if constexpr (DT) {
    // workgroup minimum -> one atomic per workgroup
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) my_min = fmin(my_min, __shfl_xor(my_min, off));
    if ((tid & 63) == 0) sred[tid >> 6] = my_min;
    __syncthreads();
    if (tid == 0) {
      double m = sred[0];
      for (int w = 1; w < NT / 64; ++w) m = fmin(m, sred[w]);
      atomicMin(a.dtmin + blockIdx.x % DT_SLOTS, (unsigned long long)__double_as_longlong(m));
    }
  }
}

}  // namespace cfd
