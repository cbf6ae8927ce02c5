// Laminar viscous residual: geometry set-up, pseudo-nodes, Green's-theorem
// face gradients and the viscous flux divergence (see viscous.h).
#include <hip/hip_runtime.h>

#include "cfd_internal.h"
#include "viscous.h"

namespace cfd {

namespace {

__device__ __forceinline__ long long node_index(const BlockDev& B, int i, int j, int k) {
  return B.node0 + ((long long)k * (B.nj + 1) + j) * (long long)(B.ni + 1) + i;
}

__device__ __forceinline__ bool cell_coords(const BlockDev& B, long long c, int& i, int& j, int& k) {
  if (c >= (long long)B.ni * B.nj * B.nk) return false;
  i = (int)(c % B.ni);
  const long long r = c / B.ni;
  j = (int)(r % B.nj);
  k = (int)(r / B.nj);
  return true;
}

// Mean of the 2 (2D) or 4 (3D) nodes of the boundary face `face` of block B
// at tangential cell coordinates (t1, t2).
template <int DIM>
__device__ void face_center(const ViscArgs& a, const BlockDev& B, int face, int t1, int t2, double* fc) {
  const int axis = face >> 1;
  const int n = axis == 0 ? B.ni : (axis == 1 ? B.nj : B.nk);
  const int ta = axis == 0 ? 1 : 0, tb = axis == 2 ? 1 : 2;
#pragma unroll
  for (int c = 0; c < DIM; ++c) fc[c] = 0.0;
#pragma unroll
  for (int o1 = 0; o1 < 2; ++o1) {
#pragma unroll
    for (int o2 = 0; o2 < (DIM == 3 ? 2 : 1); ++o2) {
      int x[3] = {0, 0, 0};
      x[axis] = (face & 1) ? n : 0;
      x[ta] = t1 + o1;
      if (DIM == 3) x[tb] = t2 + o2;
      const long long nn = node_index(B, x[0], x[1], x[2]);
#pragma unroll
      for (int c = 0; c < DIM; ++c) fc[c] += a.nodes[c * B.nnode_total + nn];
    }
  }
#pragma unroll
  for (int c = 0; c < DIM; ++c) fc[c] *= (DIM == 3 ? 0.25 : 0.5);
}

template <int DIM>
__global__ void __launch_bounds__(256) cell_centers_kernel(ViscArgs a) {
  const BlockDev B = a.blocks[blockIdx.y];
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (!cell_coords(B, c, i, j, k)) return;
  double x[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) x[d] = 0.0;
#pragma unroll
  for (int ok = 0; ok < (DIM == 3 ? 2 : 1); ++ok)
#pragma unroll
    for (int oj = 0; oj < 2; ++oj)
#pragma unroll
      for (int oi = 0; oi < 2; ++oi) {
        const long long nn = node_index(B, i + oi, j + oj, k + ok);
#pragma unroll
        for (int d = 0; d < DIM; ++d) x[d] += a.nodes[d * B.nnode_total + nn];
      }
  double* C = a.centers + B.corigin + pidx(B, i, j, k);
#pragma unroll
  for (int d = 0; d < DIM; ++d) C[d * B.vstride] = x[d] * (DIM == 3 ? 0.125 : 0.25);
}

// First ghost layer of the centres, over the chunks of transfer packs (kind 0)
// and physical patches (kind 1); layer-1 elements of a chunk are skipped.
template <int DIM>
__global__ void __launch_bounds__(CHUNK) ghost_centers_kernel(ViscArgs a) {
  using ML = MetricLayout<DIM>;
  const ChunkDev ch = a.chunks[blockIdx.x];
  if ((int)threadIdx.x >= ch.count) return;
  const int e = ch.start + threadIdx.x;
  if (ch.kind == 0) {
    const TransferDev x = a.xfers[ch.item];
    const int per_layer = x.len0 * x.len1;
    if (e >= per_layer) return;
    const int r1 = e % x.len0, r2 = e / x.len0;
    int d1, d2;
    orient_map(x.orient, r1, r2, x.dlen0, x.dlen1, d1, d2);
    const BlockDev& R = a.blocks[x.rblock];
    const BlockDev& D = a.blocks[x.dblock];
    int gi, gj, gk, si, sj, sk;
    face_cell(R, DIM, x.rface, 0, true, x.rlo0 + r1, x.rlo1 + r2, gi, gj, gk);
    face_cell(D, DIM, x.dface, 0, false, x.dlo0 + d1, x.dlo1 + d2, si, sj, sk);
    double fr[DIM], fd[DIM];
    face_center<DIM>(a, R, x.rface, x.rlo0 + r1, x.rlo1 + r2, fr);
    face_center<DIM>(a, D, x.dface, x.dlo0 + d1, x.dlo1 + d2, fd);
    const double* cd = a.centers + D.corigin + pidx(D, si, sj, sk);
    double* cg = a.centers + R.corigin + pidx(R, gi, gj, gk);
#pragma unroll
    for (int c = 0; c < DIM; ++c) cg[c * R.vstride] = fr[c] + (cd[c * D.vstride] - fd[c]);
    return;
  }
  if (ch.kind != 1) return;
  const PatchDev p = a.patches[ch.item];
  const int per_layer = p.len0 * p.len1;
  if (e >= per_layer) return;
  const int t1 = p.lo0 + e % p.len0, t2 = p.lo1 + e / p.len0;
  const BlockDev& B = a.blocks[p.block];
  int gi, gj, gk, si, sj, sk, fi, fj, fk;
  face_cell(B, DIM, p.face, 0, true, t1, t2, gi, gj, gk);
  face_cell(B, DIM, p.face, 0, false, t1, t2, si, sj, sk);
  face_cell(B, DIM, p.face, 0, (p.face & 1) != 0, t1, t2, fi, fj, fk);
  double fc[DIM], S[DIM], c0[DIM];
  face_center<DIM>(a, B, p.face, t1, t2, fc);
  const double* met = a.metric + B.morigin + pidx(B, fi, fj, fk);
  double s2 = 0.0;
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    S[c] = met[ML::S(p.face >> 1, c) * B.vstride];
    s2 += S[c] * S[c];
  }
  const double len = sqrt(s2);
  const double* cs = a.centers + B.corigin + pidx(B, si, sj, sk);
  double dn = 0.0;
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    c0[c] = cs[c * B.vstride];
    dn += (c0[c] - fc[c]) * (S[c] / len);
  }
  double* cg = a.centers + B.corigin + pidx(B, gi, gj, gk);
#pragma unroll
  for (int c = 0; c < DIM; ++c) cg[c * B.vstride] = c0[c] - 2.0 * dn * (S[c] / len);
}

// Pseudo-node (I, J, K): mean over the cells (I-1+ai, J-1+aj, K-1+ak) with at
// most one index outside the block.
template <int DIM>
__global__ void __launch_bounds__(256) pseudo_nodes_kernel(ViscArgs a, int mode) {
  constexpr int NW = DIM + 1;
  const BlockDev B = a.blocks[blockIdx.y];
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int ei = B.ni + 1, ej = B.nj + 1;
  if (n >= (long long)ei * ej * (DIM == 3 ? B.nk + 1 : 1)) return;
  const int I = (int)(n % ei);
  const long long r = n / ei;
  const int J = (int)(r % ej), K = DIM == 3 ? (int)(r / ej) : 0;
  const int nw = mode == 0 ? DIM : DIM + 1;
  double acc[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) acc[w] = 0.0;
  int cnt = 0;
#pragma unroll
  for (int ai = 0; ai < 2; ++ai)
#pragma unroll
    for (int aj = 0; aj < 2; ++aj)
#pragma unroll
      for (int ak = 0; ak < (DIM == 3 ? 2 : 1); ++ak) {
        const int out = (ai == 0 ? I == 0 : I == B.ni) + (aj == 0 ? J == 0 : J == B.nj) +
                        (DIM == 3 ? (ak == 0 ? K == 0 : K == B.nk) : 0);
        if (out > 1) continue;
        const long long p = pidx(B, I - 1 + ai, J - 1 + aj, DIM == 3 ? K - 1 + ak : 0);
        ++cnt;
        if (mode == 0) {
          const double* C = a.centers + B.corigin + p;
#pragma unroll
          for (int c = 0; c < DIM; ++c) acc[c] += C[c * B.vstride];
        } else {
          const double* q = a.q + B.origin + p;
#pragma unroll
          for (int c = 0; c < DIM; ++c) acc[c] += q[(1 + c) * B.vstride];
          acc[DIM] += a.gamma * q[(DIM + 1) * B.vstride] / q[0];
        }
      }
  const long long nn = node_index(B, I, J, K);
  double* out = mode == 0 ? a.npos : a.nval;
  for (int w = 0; w < nw; ++w) out[w * B.nnode_total + nn] = acc[w] / (double)cnt;
}

// Green's-theorem gradient of (u.., T) on one face from its dual volume:
// cell centres CL, CR with values VL, VR and the face's pseudo-nodes P[m]
// with values W[m] (2 in 2D, 4 in cyclic order in 3D).  G[v][x] = dV_v/dx.
template <int DIM>
__device__ void dual_gradient(const double* CL, const double* CR, const double* VL, const double* VR,
                              const double (*P)[DIM], const double (*W)[DIM + 1], double (*G)[DIM]) {
  constexpr int NW = DIM + 1;
#pragma unroll
  for (int v = 0; v < NW; ++v)
#pragma unroll
    for (int x = 0; x < DIM; ++x) G[v][x] = 0.0;
  if constexpr (DIM == 2) {
    const double* pos[4] = {CL, P[0], CR, P[1]};
    const double* val[4] = {VL, W[0], VR, W[1]};
    double A = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double* pa = pos[k];
      const double* pb = pos[(k + 1) % 4];
      A += 0.5 * (pa[0] * pb[1] - pb[0] * pa[1]);
      const double mx = pb[1] - pa[1], my = -(pb[0] - pa[0]);
#pragma unroll
      for (int v = 0; v < NW; ++v) {
        const double avg = 0.5 * (val[k][v] + val[(k + 1) % 4][v]);
        G[v][0] += avg * mx;
        G[v][1] += avg * my;
      }
    }
#pragma unroll
    for (int v = 0; v < NW; ++v)
#pragma unroll
      for (int x = 0; x < DIM; ++x) G[v][x] /= A;
  } else {
    double V = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int kb = (k + 1) % 4;
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        // (CR, P_k, P_k+1) and (CL, P_k+1, P_k)
        const double* pc = side == 0 ? CR : CL;
        const double* p1 = side == 0 ? P[k] : P[kb];
        const double* p2 = side == 0 ? P[kb] : P[k];
        const double* vc = side == 0 ? VR : VL;
        const double* v1 = side == 0 ? W[k] : W[kb];
        const double* v2 = side == 0 ? W[kb] : W[k];
        const double e1[3] = {p1[0] - pc[0], p1[1] - pc[1], p1[2] - pc[2]};
        const double e2[3] = {p2[0] - pc[0], p2[1] - pc[1], p2[2] - pc[2]};
        const double S[3] = {0.5 * (e1[1] * e2[2] - e1[2] * e2[1]), 0.5 * (e1[2] * e2[0] - e1[0] * e2[2]),
                             0.5 * (e1[0] * e2[1] - e1[1] * e2[0])};
        double cdot = 0.0;
#pragma unroll
        for (int x = 0; x < 3; ++x) cdot += ((pc[x] + p1[x] + p2[x]) / 3.0) * S[x];
        V += cdot / 3.0;
#pragma unroll
        for (int v = 0; v < NW; ++v) {
          const double avg = (vc[v] + v1[v] + v2[v]) / 3.0;
#pragma unroll
          for (int x = 0; x < 3; ++x) G[v][x] += avg * S[x];
        }
      }
    }
#pragma unroll
    for (int v = 0; v < NW; ++v)
#pragma unroll
      for (int x = 0; x < DIM; ++x) G[v][x] /= V;
  }
}

// Viscous flux F_v . S (momentum.., energy) from the face gradient G, the face
// velocity uf and the area vector S.
template <int DIM>
__device__ void viscous_flux(const double (*G)[DIM], const double* uf, const double* S, double mu, double kcond,
                             double* F) {
  double div = 0.0;
#pragma unroll
  for (int i = 0; i < DIM; ++i) div += G[i][i];
  double tau[DIM][DIM];
#pragma unroll
  for (int i = 0; i < DIM; ++i)
#pragma unroll
    for (int j = 0; j < DIM; ++j) tau[i][j] = mu * (G[i][j] + G[j][i]) - (i == j ? 2.0 / 3.0 * mu * div : 0.0);
  double energy = 0.0;
#pragma unroll
  for (int j = 0; j < DIM; ++j) {
    double th = 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i) th += uf[i] * tau[i][j];
    th += kcond * G[DIM][j];
    energy += th * S[j];
  }
#pragma unroll
  for (int i = 0; i < DIM; ++i) {
    double m = 0.0;
#pragma unroll
    for (int j = 0; j < DIM; ++j) m += tau[i][j] * S[j];
    F[i] = m;
  }
  F[DIM] = energy;
}

template <int DIM>
__device__ __forceinline__ void cell_values(const ViscArgs& a, const BlockDev& B, long long p, double gamma, double* V) {
  const double* q = a.q + B.origin + p;
#pragma unroll
  for (int c = 0; c < DIM; ++c) V[c] = q[(1 + c) * B.vstride];
  V[DIM] = gamma * q[(DIM + 1) * B.vstride] / q[0];
}

template <int DIM>
__global__ void __launch_bounds__(256) viscous_kernel(ViscArgs a) {
  using ML = MetricLayout<DIM>;
  constexpr int NW = DIM + 1;
  constexpr int NP = DIM == 3 ? 4 : 2;
  const BlockDev B = a.blocks[blockIdx.y];
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int i, j, k;
  if (!cell_coords(B, c, i, j, k)) return;
  const long long vs = B.vstride;
  const double* met = a.metric + B.morigin;
  double acc[NW];
#pragma unroll
  for (int v = 0; v < NW; ++v) acc[v] = 0.0;
  // one face at a time (loops not unrolled) keeps a single face's dual volume live
#pragma unroll 1
  for (int d = 0; d < DIM; ++d) {
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      // face index f = idx_d + s along d; cells f-1 (L) and f (R)
      const int di = d == 0, dj = d == 1, dk = d == 2;
      const int ri = i + di * s, rj = j + dj * s, rk = k + dk * s;
      const long long pr = pidx(B, ri, rj, rk), pl = pidx(B, ri - di, rj - dj, rk - dk);
      double CL[DIM], CR[DIM], VL[NW], VR[NW], S[DIM];
#pragma unroll
      for (int x = 0; x < DIM; ++x) {
        CL[x] = a.centers[B.corigin + x * vs + pl];
        CR[x] = a.centers[B.corigin + x * vs + pr];
        S[x] = met[ML::S(d, x) * vs + pr];
      }
      cell_values<DIM>(a, B, pl, a.gamma, VL);
      cell_values<DIM>(a, B, pr, a.gamma, VR);
      double P[NP][DIM], W[NP][NW];
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        // cyclic order over the tangential offsets (o1, o2): (0,0) (1,0) (1,1) (0,1),
        // tangential axes in increasing order
        const int o1 = (m == 1 || m == 2) ? 1 : 0, o2 = m >= 2 ? 1 : 0;
        const int ni_ = ri + (d == 0 ? 0 : o1);
        const int nj_ = rj + (d == 0 ? o1 : (d == 1 ? 0 : o2));
        const int nk_ = DIM == 3 ? rk + (d == 2 ? 0 : o2) : 0;
        const long long nn = node_index(B, ni_, nj_, nk_);
#pragma unroll
        for (int x = 0; x < DIM; ++x) P[m][x] = a.npos[x * B.nnode_total + nn];
#pragma unroll
        for (int v = 0; v < NW; ++v) W[m][v] = a.nval[v * B.nnode_total + nn];
      }
      double G[NW][DIM], uf[DIM], F[NW];
      dual_gradient<DIM>(CL, CR, VL, VR, P, W, G);
#pragma unroll
      for (int x = 0; x < DIM; ++x) uf[x] = 0.5 * (VL[x] + VR[x]);
      viscous_flux<DIM>(G, uf, S, a.mu, a.kcond, F);
#pragma unroll
      for (int v = 0; v < NW; ++v) acc[v] += s ? F[v] : -F[v];
    }
  }
  const double iv = met[ML::INVVOL * vs + pidx(B, i, j, k)];
#pragma unroll
  for (int v = 0; v < NW; ++v) a.rv[v * B.ncell_total + B.packed + c] = acc[v] * iv;
}

dim3 grid_of(long long items, int nblocks) { return dim3((unsigned)((items + 255) / 256), (unsigned)nblocks); }

}  // namespace

hipError_t launch_cell_centers(int dim, const ViscArgs& a, long long max_cells, int nblocks, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(cell_centers_kernel<2>, grid_of(max_cells, nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(cell_centers_kernel<3>, grid_of(max_cells, nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_ghost_centers(int dim, const ViscArgs& a, int nchunks, hipStream_t s) {
  if (nchunks <= 0) return hipSuccess;
  if (dim == 2)
    hipLaunchKernelGGL(ghost_centers_kernel<2>, dim3(nchunks), dim3(CHUNK), 0, s, a);
  else
    hipLaunchKernelGGL(ghost_centers_kernel<3>, dim3(nchunks), dim3(CHUNK), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pseudo_nodes(int dim, const ViscArgs& a, int mode, long long max_nodes, int nblocks, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(pseudo_nodes_kernel<2>, grid_of(max_nodes, nblocks), dim3(256), 0, s, a, mode);
  else
    hipLaunchKernelGGL(pseudo_nodes_kernel<3>, grid_of(max_nodes, nblocks), dim3(256), 0, s, a, mode);
  return hipGetLastError();
}

hipError_t launch_viscous(int dim, const ViscArgs& a, long long max_cells, int nblocks, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(viscous_kernel<2>, grid_of(max_cells, nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(viscous_kernel<3>, grid_of(max_cells, nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace cfd
