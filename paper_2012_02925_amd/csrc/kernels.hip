// Device kernels of the Euler hot path and their host-side launchers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "cfd_internal.h"
#include "device_math.h"
#include "kernels.h"
#include "stage_launch.h"

namespace cfd {

// ---------------------------------------------------------------------------
// ghost fill: pack / physical patches / unpack (Sec. 2 ghost cells; Sec. 7.2
// V1 pack/unpack and V5 persistent per-connection buffers), or, for blocks
// on the same GPU, connected ghosts filled directly by copying the donor's
// interior (Sec. 5: self-connected ghosts are filled by copying) in the same
// launch as the physical patches

template <int DIM>
__device__ __forceinline__ void mirror_velocity(double* q, const double* S) {
  double s2 = 0.0, un = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    s2 += S[d] * S[d];
    un += q[1 + d] * S[d];
  }
  const double f = 2.0 * un / s2;  // 2 (u . n) n with n = S/|S|
#pragma unroll
  for (int d = 0; d < DIM; ++d) q[1 + d] -= f * S[d];
}

// Characteristic boundary states (Sec. 2 names the boundary types; the forms
// are the textbook ones).  g holds the primitive state of the interior cell
// next to the face on entry and the boundary state on return; n is the unit
// normal pointing out of the block.
//
// Farfield: Riemann invariants R+ = V_i + 2 c_i/(gamma-1) from the interior
// and R- = V_inf - 2 c_inf/(gamma-1) from the free stream qf give the normal
// velocity (R+ + R-)/2 and the sound speed (gamma-1)(R+ - R-)/4; entropy
// p/rho^gamma and tangential velocity come from the upwind side.  Supersonic
// inflow takes qf, supersonic outflow keeps the interior state.
template <int DIM>
__device__ void farfield_state(double* g, const double* n, const double* qf, const Gas& gs) {
  constexpr int NV = DIM + 2;
  double Vi = 0.0, Vf = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    Vi += g[1 + d] * n[d];
    Vf += qf[1 + d] * n[d];
  }
  const double ci = sqrt(gs.gamma * g[NV - 1] / g[0]);
  const double cf = sqrt(gs.gamma * qf[NV - 1] / qf[0]);
  if (Vf <= -cf) {
#pragma unroll
    for (int v = 0; v < NV; ++v) g[v] = qf[v];
    return;
  }
  if (Vi >= ci) return;
  const double Rp = Vi + 2.0 * ci / gs.gm1;
  const double Rm = Vf - 2.0 * cf / gs.gm1;
  const double Vb = 0.5 * (Rp + Rm);
  const double cb = 0.25 * gs.gm1 * (Rp - Rm);
  double side[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) side[v] = Vb >= 0.0 ? g[v] : qf[v];
  const double s = side[NV - 1] / pow(side[0], gs.gamma);
  const double rb = pow(cb * cb / (gs.gamma * s), 1.0 / gs.gm1);
  double us = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) us += side[1 + d] * n[d];
  g[0] = rb;
#pragma unroll
  for (int d = 0; d < DIM; ++d) g[1 + d] = side[1 + d] - us * n[d] + Vb * n[d];
  g[NV - 1] = rb * cb * cb / gs.gamma;
}

// Subsonic inflow with stagnation pressure p0, stagnation density rho0 and
// unit direction d (P = p0, rho0, d): static pressure from the interior,
// capped at p0; density and speed from the isentropic relations.
template <int DIM>
__device__ void subsonic_inflow_state(double* g, const double* P, const Gas& gs) {
  constexpr int NV = DIM + 2;
  const double p0 = P[0], r0 = P[1];
  const double pb = fmin(g[NV - 1], p0);
  const double rb = r0 * pow(pb / p0, 1.0 / gs.gamma);
  const double sp = sqrt(fmax(2.0 * gs.gamma / gs.gm1 * (p0 / r0 - pb / rb), 0.0));
  g[0] = rb;
#pragma unroll
  for (int d = 0; d < DIM; ++d) g[1 + d] = sp * P[2 + d];
  g[NV - 1] = pb;
}

// Subsonic outflow: the back pressure replaces the interior pressure unless
// the outflow is supersonic.
template <int DIM>
__device__ void subsonic_outflow_state(double* g, const double* n, double pback, const Gas& gs) {
  constexpr int NV = DIM + 2;
  double Vi = 0.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) Vi += g[1 + d] * n[d];
  if (Vi < sqrt(gs.gamma * g[NV - 1] / g[0])) g[NV - 1] = pback;
}

// dt <- cfl * min over the DT_SLOTS slots (when promote); slots <- +inf.
// Called by one whole wavefront (lanes 0..63): every lane reads one slot, the
// minimum is formed by shuffles, and each lane resets its own slot after that.
__device__ __forceinline__ void promote_slots(double* dt, unsigned long long* dtmin, double cfl, int promote,
                                              double* out) {
  static_assert(DT_SLOTS == 64, "one slot per lane of the wavefront");
  const int t = threadIdx.x;
  double m = __longlong_as_double((long long)dtmin[t]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmin(m, __shfl_xor(m, off));
  if (t == 0) {
    if (promote) dt[0] = cfl * m;
    if (out) out[0] = cfl * m;
  }
  if (promote) dtmin[t] = (unsigned long long)__double_as_longlong(INFINITY);
}

template <int DIM>
__global__ void __launch_bounds__(CHUNK) ghost_kernel(GhostArgs a) {
  constexpr int NV = DIM + 2;
  using ML = MetricLayout<DIM>;
  if (a.dtmin && blockIdx.x == 0 && threadIdx.x < 64) promote_slots(a.dt, a.dtmin, a.cfl, 1, nullptr);
  const ChunkDev ch = a.chunks[a.chunk_begin + blockIdx.x];
  const int e = ch.start + threadIdx.x;
  if (threadIdx.x >= ch.count) return;
  if (ch.kind == 3) {
    // direct copy of a connection (same GPU): the donor's interior layer
    // `layer` at the mapped position straight into the receiver's ghost
    // layer, the composition of the pack and unpack below without the buffer
    const TransferDev x = a.xfers[ch.item];
    const int layer = e & 1;
    const int r = e >> 1;
    const int r1 = r % x.len0, r2 = r / x.len0;
    int d1, d2;
    orient_map(x.orient, r1, r2, x.dlen0, x.dlen1, d1, d2);
    const BlockDev& D = a.blocks[x.dblock];
    const BlockDev& R = a.blocks[x.rblock];
    int i, j, k, gi, gj, gk;
    face_cell(D, DIM, x.dface, layer, false, x.dlo0 + d1, x.dlo1 + d2, i, j, k);
    face_cell(R, DIM, x.rface, layer, true, x.rlo0 + r1, x.rlo1 + r2, gi, gj, gk);
    const double* qd = a.q + D.origin + pidx(D, i, j, k);
    double* qr = a.q + R.origin + pidx(R, gi, gj, gk);
    double val[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) val[v] = qd[v * D.vstride];
#pragma unroll
    for (int v = 0; v < NV; ++v) qr[v * R.vstride] = val[v];
    return;
  }
  if (ch.kind == 0 || ch.kind == 2) {
    const TransferDev x = a.xfers[ch.item];
    const int per_layer = x.len0 * x.len1;
    const int cnt = 2 * per_layer;
    // the two layers of one face position are neighbouring elements (on an
    // i-face the two cells share a cache line, so they go to adjacent lanes)
    const int layer = e & 1;
    const int r = e >> 1;
    const int r1 = r % x.len0, r2 = r / x.len0;
    double* seg = a.buf + x.buf;
    if (ch.kind == 0) {
      int d1, d2;
      orient_map(x.orient, r1, r2, x.dlen0, x.dlen1, d1, d2);
      const BlockDev& B = a.blocks[x.dblock];
      int i, j, k;
      face_cell(B, DIM, x.dface, layer, false, x.dlo0 + d1, x.dlo1 + d2, i, j, k);
      const double* q = a.q + B.origin + pidx(B, i, j, k);
#pragma unroll
      for (int v = 0; v < NV; ++v) seg[v * cnt + e] = q[v * B.vstride];
    } else {
      const BlockDev& B = a.blocks[x.rblock];
      int i, j, k;
      face_cell(B, DIM, x.rface, layer, true, x.rlo0 + r1, x.rlo1 + r2, i, j, k);
      double* q = a.q + B.origin + pidx(B, i, j, k);
#pragma unroll
      for (int v = 0; v < NV; ++v) q[v * B.vstride] = seg[v * cnt + e];
    }
    return;
  }
  // physical patch
  const PatchDev p = a.patches[ch.item];
  const int layer = e & 1;  // (layers of one face position side by side, as above)
  const int r = e >> 1;
  const int t1 = p.lo0 + r % p.len0, t2 = p.lo1 + r / p.len0;
  const BlockDev& B = a.blocks[p.block];
  const long long vs = B.vstride;
  int gi, gj, gk;
  face_cell(B, DIM, p.face, layer, true, t1, t2, gi, gj, gk);
  double* base = a.q + B.origin;
  double g[NV];
  if (p.kind == PK_SUP_INFLOW) {
#pragma unroll
    for (int v = 0; v < NV; ++v) g[v] = a.bcparams[p.param * MAXV + v];
  } else {
    int si, sj, sk;
    const bool mirror = p.kind == PK_SLIP_WALL || p.kind == PK_NOSLIP_WALL;
    face_cell(B, DIM, p.face, mirror ? layer : 0, false, t1, t2, si, sj, sk);
    const long long s = pidx(B, si, sj, sk);
#pragma unroll
    for (int v = 0; v < NV; ++v) g[v] = base[v * vs + s];
    if (p.kind == PK_NOSLIP_WALL) {
      // adiabatic no-slip wall: velocity negated, rho and p (so T) copied
#pragma unroll
      for (int d = 0; d < DIM; ++d) g[1 + d] = -g[1 + d];
    } else if (p.kind == PK_SUB_INFLOW) {
      subsonic_inflow_state<DIM>(g, a.bcparams + p.param * MAXV, a.gas);
    } else if (p.kind != PK_EXTRAP_OUTFLOW) {
      // area vector of the boundary face itself
      int fi, fj, fk;
      face_cell(B, DIM, p.face, 0, (p.face & 1) != 0, t1, t2, fi, fj, fk);
      const long long fidx = pidx(B, fi, fj, fk);
      const double* met = a.metric + B.morigin;
      double S[DIM];
#pragma unroll
      for (int c = 0; c < DIM; ++c) S[c] = met[ML::S(p.face >> 1, c) * vs + fidx];
      if (p.kind == PK_SLIP_WALL) {
        mirror_velocity<DIM>(g, S);
      } else {
        double s2 = 0.0, n[DIM];
#pragma unroll
        for (int c = 0; c < DIM; ++c) s2 += S[c] * S[c];
        const double len = sqrt(s2);
#pragma unroll
        for (int c = 0; c < DIM; ++c) n[c] = (p.face & 1) ? S[c] / len : -(S[c] / len);
        if (p.kind == PK_FARFIELD)
          farfield_state<DIM>(g, n, a.bcparams + p.param * MAXV, a.gas);
        else
          subsonic_outflow_state<DIM>(g, n, a.bcparams[p.param * MAXV], a.gas);
      }
    }
  }
  const long long gidx = pidx(B, gi, gj, gk);
#pragma unroll
  for (int v = 0; v < NV; ++v) base[v * vs + gidx] = g[v];
}

// ---------------------------------------------------------------------------
// per-cell kernels over the packed layout (grid.y = block)

__device__ __forceinline__ bool cell_of(const BlockDev& B, long long c, int& i, int& j, int& k) {
  const long long n = (long long)B.ni * B.nj * B.nk;
  if (c >= n) return false;
  i = (int)(c % B.ni);
  const long long r = c / B.ni;
  j = (int)(r % B.nj);
  k = (int)(r / B.nj);
  return true;
}

template <int DIM>
__global__ void set_state_kernel(CellArgs a) {
  constexpr int NV = DIM + 2;
  const BlockDev B = a.blocks[blockIdx.y];
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (!cell_of(B, c, i, j, k)) return;
  double in[NV], q[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) in[v] = a.src[v * B.ncell_total + B.packed + c];
  if (a.flag_primitive) {
#pragma unroll
    for (int v = 0; v < NV; ++v) q[v] = in[v];
  } else {
    cons_to_prim<DIM>(in, a.gas, q);
  }
  bool ok = q[0] > 0.0 && q[NV - 1] > 0.0 && isfinite(q[0]) && isfinite(q[NV - 1]);
#pragma unroll
  for (int v = 1; v < NV - 1; ++v) ok = ok && isfinite(q[v]);
  if (!ok) atomicOr(a.err, 1);
  double* dst = a.dst + B.origin + pidx(B, i, j, k);
#pragma unroll
  for (int v = 0; v < NV; ++v) dst[v * B.vstride] = q[v];
}

template <int DIM>
__global__ void get_state_kernel(CellArgs a) {
  constexpr int NV = DIM + 2;
  const BlockDev B = a.blocks[blockIdx.y];
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (!cell_of(B, c, i, j, k)) return;
  const double* src = a.src + B.origin + pidx(B, i, j, k);
  double q[NV], Q[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) q[v] = src[v * B.vstride];
  if (a.flag_primitive) {
#pragma unroll
    for (int v = 0; v < NV; ++v) Q[v] = q[v];
  } else {
    prim_to_cons<DIM>(q, a.gas, Q);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) a.dst[v * B.ncell_total + B.packed + c] = Q[v];
}

// Omega / lambda of every interior cell, reduced to one minimum (bits of a
// positive double, atomicMin on the unsigned pattern is an exact min).
template <int DIM>
__global__ void __launch_bounds__(256) cell_dt_kernel(CellArgs a) {
  constexpr int NV = DIM + 2;
  using ML = MetricLayout<DIM>;
  __shared__ double red[4];
  const BlockDev B = a.blocks[blockIdx.y];
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double m = 1.0e300;
  int i, j, k;
  if (cell_of(B, c, i, j, k)) {
    const long long ci = pidx(B, i, j, k);
    const double* q = a.src + B.origin + ci;
    const double* met = a.metric + B.morigin + ci;
    const long long vs = B.vstride;
    double w[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v] = q[v * vs];
    const double cs = sqrt(a.gas.gamma * w[NV - 1] / w[0]);
    double lam = 0.0, s2sum = 0.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const long long step = d == 0 ? 1 : (d == 1 ? (long long)B.pi : (long long)B.pi * B.pj);
      double un = 0.0, s2 = 0.0;
#pragma unroll
      for (int cc = 0; cc < DIM; ++cc) {
        const double sb = 0.5 * (met[ML::S(d, cc) * vs] + met[ML::S(d, cc) * vs + step]);
        un += w[1 + cc] * sb;
        s2 += sb * sb;
      }
      lam += fabs(un) + cs * sqrt(s2);
      s2sum += s2;
    }
    if (a.visc_cv > 0.0) lam += a.visc_cv / w[0] * s2sum * met[ML::INVVOL * vs];
    m = 1.0 / (lam * met[ML::INVVOL * vs]);
    if (a.dtloc) a.dtloc[B.packed + c] = a.cfl * m;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmin(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
    const unsigned w = blockIdx.y * gridDim.x + blockIdx.x;
    atomicMin(a.dtmin + w % DT_SLOTS, (unsigned long long)__double_as_longlong(r));
  }
}

__global__ void __launch_bounds__(64) dt_promote_kernel(double* dt, unsigned long long* dtmin, double cfl, int promote,
                                                        double* out) {
  promote_slots(dt, dtmin, cfl, promote, out);
}

__global__ void set_u64_kernel(unsigned long long* p, unsigned long long v, int n) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) p[t] = v;
}

__global__ void copy_dt_kernel(const double* src, double* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) dst[0] = src[0];
}

// ---------------------------------------------------------------------------
// metrics from nodes (setup)

__device__ __forceinline__ void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

template <int DIM>
__global__ void metrics_kernel(MetricArgs a) {
  using ML = MetricLayout<DIM>;
  const BlockDev B = a.blocks[blockIdx.y];
  // positions (i, j, k) in [0, ni] x [0, nj] x [0, nk] (k = 0 only in 2D)
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ei = B.ni + 1, ej = B.nj + 1, ek = DIM == 3 ? B.nk + 1 : 1;
  if (c >= (long long)ei * ej * ek) return;
  const int i = (int)(c % ei);
  const int j = (int)((c / ei) % ej);
  const int k = (int)(c / ((long long)ei * ej));
  const long long nn = B.nnode_total;
  const int ni1 = B.ni + 1, nj1 = B.nj + 1;
  auto X = [&](int cc, int ii, int jj, int kk) -> double {
    return a.nodes[cc * nn + B.node0 + ((long long)kk * nj1 + jj) * ni1 + ii];
  };
  double* met = a.metric + B.morigin;
  const long long vs = B.vstride;
  const long long ci = pidx(B, i, j, k);
  if constexpr (DIM == 2) {
    if (j < B.nj) {  // i-face from node (i,j) to (i,j+1)
      const double dx = X(0, i, j + 1, 0) - X(0, i, j, 0), dy = X(1, i, j + 1, 0) - X(1, i, j, 0);
      met[ML::S(0, 0) * vs + ci] = dy;
      met[ML::S(0, 1) * vs + ci] = -dx;
    }
    if (i < B.ni) {  // j-face from node (i,j) to (i+1,j)
      const double dx = X(0, i + 1, j, 0) - X(0, i, j, 0), dy = X(1, i + 1, j, 0) - X(1, i, j, 0);
      met[ML::S(1, 0) * vs + ci] = -dy;
      met[ML::S(1, 1) * vs + ci] = dx;
    }
    if (i < B.ni && j < B.nj) {
      const double d1x = X(0, i + 1, j + 1, 0) - X(0, i, j, 0), d1y = X(1, i + 1, j + 1, 0) - X(1, i, j, 0);
      const double d2x = X(0, i, j + 1, 0) - X(0, i + 1, j, 0), d2y = X(1, i, j + 1, 0) - X(1, i + 1, j, 0);
      const double vol = 0.5 * (d1x * d2y - d1y * d2x);
      if (!(vol > 0.0) || !isfinite(vol)) atomicOr(a.err, 1);
      met[ML::INVVOL * vs + ci] = 1.0 / vol;
    }
  } else {
    auto P = [&](int ii, int jj, int kk, double* p) {
      p[0] = X(0, ii, jj, kk);
      p[1] = X(1, ii, jj, kk);
      p[2] = X(2, ii, jj, kk);
    };
    // area vector 1/2 (c - a) x (d - b) of quad a b c d, plus the mean node
    auto quad = [&](const double* pa, const double* pb, const double* pc, const double* pd, double* S, double* m) {
      double u[3], w[3];
      for (int q = 0; q < 3; ++q) {
        u[q] = pc[q] - pa[q];
        w[q] = pd[q] - pb[q];
        m[q] = 0.25 * (pa[q] + pb[q] + pc[q] + pd[q]);
      }
      cross3(u, w, S);
      for (int q = 0; q < 3; ++q) S[q] *= 0.5;
    };
    double pa[3], pb[3], pc[3], pd[3], S[3], m[3];
    if (j < B.nj && k < B.nk) {  // i-face: (i,j,k) (i,j+1,k) (i,j+1,k+1) (i,j,k+1)
      P(i, j, k, pa); P(i, j + 1, k, pb); P(i, j + 1, k + 1, pc); P(i, j, k + 1, pd);
      quad(pa, pb, pc, pd, S, m);
      for (int q = 0; q < 3; ++q) met[ML::S(0, q) * vs + ci] = S[q];
    }
    if (i < B.ni && k < B.nk) {  // j-face: (i,j,k) (i,j,k+1) (i+1,j,k+1) (i+1,j,k)
      P(i, j, k, pa); P(i, j, k + 1, pb); P(i + 1, j, k + 1, pc); P(i + 1, j, k, pd);
      quad(pa, pb, pc, pd, S, m);
      for (int q = 0; q < 3; ++q) met[ML::S(1, q) * vs + ci] = S[q];
    }
    if (i < B.ni && j < B.nj) {  // k-face: (i,j,k) (i+1,j,k) (i+1,j+1,k) (i,j+1,k)
      P(i, j, k, pa); P(i + 1, j, k, pb); P(i + 1, j + 1, k, pc); P(i, j + 1, k, pd);
      quad(pa, pb, pc, pd, S, m);
      for (int q = 0; q < 3; ++q) met[ML::S(2, q) * vs + ci] = S[q];
    }
    if (i < B.ni && j < B.nj && k < B.nk) {
      // volume = 1/3 sum_f xbar_f . S_f (outward); low faces enter with a minus sign
      double vol = 0.0;
      for (int d = 0; d < 3; ++d) {
        for (int side = 0; side < 2; ++side) {
          const int ii = i + (d == 0 ? side : 0), jj = j + (d == 1 ? side : 0), kk = k + (d == 2 ? side : 0);
          if (d == 0) {
            P(ii, jj, kk, pa); P(ii, jj + 1, kk, pb); P(ii, jj + 1, kk + 1, pc); P(ii, jj, kk + 1, pd);
          } else if (d == 1) {
            P(ii, jj, kk, pa); P(ii, jj, kk + 1, pb); P(ii + 1, jj, kk + 1, pc); P(ii + 1, jj, kk, pd);
          } else {
            P(ii, jj, kk, pa); P(ii + 1, jj, kk, pb); P(ii + 1, jj + 1, kk, pc); P(ii, jj + 1, kk, pd);
          }
          quad(pa, pb, pc, pd, S, m);
          const double f = m[0] * S[0] + m[1] * S[1] + m[2] * S[2];
          vol += side ? f : -f;
        }
      }
      vol *= (1.0 / 3.0);
      if (!(vol > 0.0) || !isfinite(vol)) atomicOr(a.err, 1);
      met[ML::INVVOL * vs + ci] = 1.0 / vol;
    }
  }
}

// padded export of a state buffer: block after block, [var][k+2][j+2][i+2]
template <int DIM>
__global__ void export_padded_kernel(CellArgs a) {
  constexpr int NV = DIM + 2;
  const BlockDev B = a.blocks[blockIdx.y];
  const int ei = B.ni + 4, ej = B.nj + 4, ek = DIM == 3 ? B.nk + 4 : 1;
  const long long n = (long long)ei * ej * ek;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int i = (int)(c % ei) - 2;
  const int j = (int)((c / ei) % ej) - 2;
  const int k = (int)(c / ((long long)ei * ej)) - (DIM == 3 ? 2 : 0);
  const double* src = a.src + B.origin + pidx(B, i, j, k);
  double* dst = a.dst + a.offsets[blockIdx.y];
#pragma unroll
  for (int v = 0; v < NV; ++v) dst[v * n + c] = src[v * B.vstride];
}

// ---------------------------------------------------------------------------
// residual norms: per-part sums of squares over fixed contiguous cell ranges,
// then one workgroup adds the parts in order

template <int NV>
__global__ void __launch_bounds__(256) sumsq_partial_kernel(const double* R, long long ncells, double* partial) {
  __shared__ double red[256];
  const long long per = (ncells + gridDim.x - 1) / gridDim.x;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = min(ncells, lo + per);
  for (int v = 0; v < NV; ++v) {
    double s = 0.0;
    for (long long c = lo + threadIdx.x; c < hi; c += blockDim.x) s += R[v * ncells + c] * R[v * ncells + c];
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

template <int NV>
__global__ void __launch_bounds__(256) norms_kernel(const double* partial, int nparts, long long ncells,
                                                    double* norms) {
  __shared__ double red[256];
  for (int v = 0; v < NV; ++v) {
    double s = 0.0;
    for (int p = threadIdx.x; p < nparts; p += blockDim.x) s += partial[(long long)v * nparts + p];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) norms[v] = sqrt(red[0] / (double)ncells);
    __syncthreads();
  }
}

hipError_t launch_sumsq(int nvar, const double* R, long long ncells, double* partial, int nparts,
                        double* norms, hipStream_t s) {
  if (nvar == 4) {
    hipLaunchKernelGGL(sumsq_partial_kernel<4>, dim3(nparts), dim3(256), 0, s, R, ncells, partial);
    hipLaunchKernelGGL(norms_kernel<4>, dim3(1), dim3(256), 0, s, partial, nparts, ncells, norms);
  } else {
    hipLaunchKernelGGL(sumsq_partial_kernel<5>, dim3(nparts), dim3(256), 0, s, R, ncells, partial);
    hipLaunchKernelGGL(norms_kernel<5>, dim3(1), dim3(256), 0, s, partial, nparts, ncells, norms);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// stage kernel variants

const StageVariant* stage_variants(int dim, int* count) {
  static const StageVariant v2[] = {{64, 4, 1}, {32, 8, 1}, {16, 16, 1}};
  static const StageVariant v3[] = {{64, 4, 32}, {32, 8, 32}, {32, 8, 64}};
  *count = 3;
  return dim == 2 ? v2 : v3;
}

hipError_t launch_stage(int dim, int flux, int lim, int variant, bool ff, const StageArgs& a, int grid,
                        bool persistent, hipStream_t s) {
  return dim == 2 ? launch_stage_2d(flux, lim, variant, ff, a, grid, persistent, s)
                  : launch_stage_3d(flux, lim, variant, ff, a, grid, persistent, s);
}

// ---------------------------------------------------------------------------
// launchers

hipError_t launch_ghost(int dim, const GhostArgs& a, int nchunks, hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  if (dim == 2)
    hipLaunchKernelGGL(ghost_kernel<2>, dim3(nchunks), dim3(CHUNK), 0, s, a);
  else
    hipLaunchKernelGGL(ghost_kernel<3>, dim3(nchunks), dim3(CHUNK), 0, s, a);
  return hipGetLastError();
}

static dim3 cell_grid(long long max_cells, int nblocks) {
  return dim3((unsigned)((max_cells + 255) / 256), (unsigned)nblocks);
}

hipError_t launch_set_state(int dim, const CellArgs& a, long long max_cells, int nblocks, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(set_state_kernel<2>, cell_grid(max_cells, nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(set_state_kernel<3>, cell_grid(max_cells, nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_get_state(int dim, const CellArgs& a, long long max_cells, int nblocks, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(get_state_kernel<2>, cell_grid(max_cells, nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(get_state_kernel<3>, cell_grid(max_cells, nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_cell_dt(int dim, const CellArgs& a, long long max_cells, int nblocks, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(cell_dt_kernel<2>, cell_grid(max_cells, nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(cell_dt_kernel<3>, cell_grid(max_cells, nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

// One thread per padded cell of a block (grid.y = block).  A cell gets the
// factor of direction d if it touches a face along d (index -1 .. n along d)
// and is interior along the other directions; every other entry is 0.
template <int DIM>
__global__ void freeze_kernel(FreezeArgs a) {
  constexpr int NV = DIM + 2;
  const BlockDev B = a.blocks[blockIdx.y];
  const int ei = B.ni + 4, ej = B.nj + 4, ek = DIM == 3 ? B.nk + 4 : 1;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= (long long)ei * ej * ek) return;
  const int i = (int)(c % ei) - 2;
  const long long r = c / ei;
  const int j = (int)(r % ej) - 2;
  const int k = DIM == 3 ? (int)(r / ej) - 2 : 0;
  const long long vs = B.vstride;
  const long long p = pidx(B, i, j, k);
  const double* q = a.q + B.origin;
  double* phi = a.phi + B.lorigin;
  const int idx[3] = {i, j, k};
  const int ext[3] = {B.ni, B.nj, B.nk};
  const long long step[3] = {1, B.pi, (long long)B.pi * B.pj};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    bool ok = idx[d] >= -1 && idx[d] <= ext[d];
#pragma unroll
    for (int e = 0; e < DIM; ++e)
      if (e != d) ok = ok && idx[e] >= 0 && idx[e] < ext[e];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double f = 0.0;
      if (ok) {
        const double q0 = q[v * vs + p];
        const double dm = q0 - q[v * vs + p - step[d]];
        const double dp = q[v * vs + p + step[d]] - q0;
        f = a.limiter == LIM_VANLEER ? frozen_factor<LIM_VANLEER>(dp, dm, 0.0)
                                     : frozen_factor<LIM_VANALBADA>(dp, dm, a.e2[v]);
      }
      phi[(d * NV + v) * vs + p] = f;
    }
  }
}

// ---------------------------------------------------------------------------
// debug checks (cfd_config.debug_flags)

// CFD_NAN_GHOSTS: quiet NaN into every cell of the ghost region (i in
// [-2, ni+2) x j in [-2, nj+2) [x k in [-2, nk+2)] minus the interior) of
// every array of a state buffer, before the ghost fill, so a ghost value the
// fill does not provide (or a corner ghost, never filled) surfaces as NaN
// wherever a kernel reads it.
template <int DIM>
__global__ void __launch_bounds__(256) nan_ghosts_kernel(CellArgs a) {
  constexpr int NV = DIM + 2;
  const BlockDev B = a.blocks[blockIdx.y];
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long ex = B.ni + 4, ey = B.nj + 4, ez = DIM == 3 ? B.nk + 4 : 1;
  if (n >= ex * ey * ez) return;
  const int i = (int)(n % ex) - 2;
  const int j = (int)((n / ex) % ey) - 2;
  const int k = DIM == 3 ? (int)(n / (ex * ey)) - 2 : 0;
  if (i >= 0 && i < B.ni && j >= 0 && j < B.nj && (DIM == 2 || (k >= 0 && k < B.nk))) return;
  double* q = a.dst + B.origin + pidx(B, i, j, k);
  const double qnan = __longlong_as_double(0x7ff8000000000000LL);
#pragma unroll
  for (int v = 0; v < NV; ++v) q[v * B.vstride] = qnan;
}

// CFD_CHECK_FINITE: flag (*a.err |= 1) an interior cell of a primitive state
// buffer whose density or pressure is not positive and finite or whose
// velocity is not finite.
template <int DIM>
__global__ void __launch_bounds__(256) check_state_kernel(CellArgs a) {
  constexpr int NV = DIM + 2;
  const BlockDev B = a.blocks[blockIdx.y];
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (!cell_of(B, c, i, j, k)) return;
  const double* q = a.src + B.origin + pidx(B, i, j, k);
  const double r = q[0], p = q[(NV - 1) * B.vstride];
  bool ok = r > 0.0 && p > 0.0 && isfinite(r) && isfinite(p);
#pragma unroll
  for (int v = 1; v < NV - 1; ++v) ok = ok && isfinite(q[v * B.vstride]);
  if (!ok) atomicOr(a.err, 1);
}

// Classical fourth-order Runge-Kutta (not in the paper; the M-stage scheme of
// Sec. 2 is the default): with the stage inputs Y2, Y3, Y4 and
// Z = Q - dt/6 R(Y4) written by the stage kernel, per interior cell in
// conservative variables
//   Q^(n+1) = Q + [(Y2 - Q) + 2 (Y3 - Q) + (Y4 - Q)] / 3 + (Z - Q)
//           = Q - dt/6 (R(Q) + 2 R(Y2) + 2 R(Y3) + R(Y4)).
// Each difference is a multiple of dt R, so a steady state stays exactly
// steady.  out may alias q (each cell reads its own values first).
template <int DIM>
__global__ void __launch_bounds__(256) rk4_combine_kernel(Rk4Args a) {
  constexpr int NV = DIM + 2;
  const BlockDev B = a.blocks[blockIdx.y];
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (!cell_of(B, c, i, j, k)) return;
  const long long p = B.origin + pidx(B, i, j, k), vs = B.vstride;
  double w[NV], Q[NV], Y[NV], acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) w[v] = a.q[v * vs + p];
  prim_to_cons<DIM>(w, a.gas, Q);
  const double* src[3] = {a.y2, a.y3, a.y4};
  const double wt[3] = {1.0, 2.0, 1.0};
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v] = src[s][v * vs + p];
    prim_to_cons<DIM>(w, a.gas, Y);
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += wt[s] * (Y[v] - Q[v]);
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) w[v] = a.z[v * vs + p];
  prim_to_cons<DIM>(w, a.gas, Y);
#pragma unroll
  for (int v = 0; v < NV; ++v) Y[v] = Q[v] + acc[v] / 3.0 + (Y[v] - Q[v]);
  cons_to_prim<DIM>(Y, a.gas, w);
#pragma unroll
  for (int v = 0; v < NV; ++v) a.out[v * vs + p] = w[v];
}

hipError_t launch_rk4_combine(int dim, const Rk4Args& a, long long max_cells, int nblocks, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(rk4_combine_kernel<2>, cell_grid(max_cells, nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(rk4_combine_kernel<3>, cell_grid(max_cells, nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

// CFD_CHECK_FINITE: flag a non-finite entry of a packed array (n doubles).
__global__ void __launch_bounds__(256) check_packed_kernel(const double* x, long long n, int* err) {
  bool ok = true;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    ok = ok && isfinite(x[e]);
  if (!ok) atomicOr(err, 1);
}

hipError_t launch_nan_ghosts(int dim, const CellArgs& a, long long max_padded, int nblocks, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(nan_ghosts_kernel<2>, cell_grid(max_padded, nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(nan_ghosts_kernel<3>, cell_grid(max_padded, nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_check_state(int dim, const CellArgs& a, long long max_cells, int nblocks, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(check_state_kernel<2>, cell_grid(max_cells, nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(check_state_kernel<3>, cell_grid(max_cells, nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_check_packed(const double* x, long long n, int* err, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long long blocks = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(check_packed_kernel, dim3((unsigned)blocks), dim3(256), 0, s, x, n, err);
  return hipGetLastError();
}

hipError_t launch_freeze(int dim, const FreezeArgs& a, long long max_padded, int nblocks, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(freeze_kernel<2>, cell_grid(max_padded, nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(freeze_kernel<3>, cell_grid(max_padded, nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_export_padded(int dim, const CellArgs& a, long long max_padded, int nblocks, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(export_padded_kernel<2>, cell_grid(max_padded, nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(export_padded_kernel<3>, cell_grid(max_padded, nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_metrics(int dim, const MetricArgs& a, long long max_pos, int nblocks, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(metrics_kernel<2>, cell_grid(max_pos, nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(metrics_kernel<3>, cell_grid(max_pos, nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_dt_promote(double* dt, unsigned long long* dtmin, double cfl, int promote, double* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(dt_promote_kernel, dim3(1), dim3(64), 0, s, dt, dtmin, cfl, promote, out);
  return hipGetLastError();
}

hipError_t launch_set_u64(unsigned long long* p, unsigned long long v, int n, hipStream_t s) {
  hipLaunchKernelGGL(set_u64_kernel, dim3(1), dim3(64), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_copy_dt(const double* src, double* dst, hipStream_t s) {
  hipLaunchKernelGGL(copy_dt_kernel, dim3(1), dim3(64), 0, s, src, dst);
  return hipGetLastError();
}

}  // namespace cfd
