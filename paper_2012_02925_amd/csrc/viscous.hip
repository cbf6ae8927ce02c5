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

// Index decode in 32-bit arithmetic (a block holds fewer than 2^31 cells and
// nodes; 64-bit division would dominate these light kernels).
__device__ __forceinline__ bool decode3(long long n, int e0, int e1, int e2, int& a0, int& a1, int& a2) {
  if (n >= (long long)e0 * e1 * e2) return false;
  const unsigned u = (unsigned)n;
  const unsigned r = u / (unsigned)e0;
  a0 = (int)(u - r * (unsigned)e0);
  a2 = (int)(r / (unsigned)e1);
  a1 = (int)(r - (unsigned)a2 * (unsigned)e1);
  return true;
}

__device__ __forceinline__ bool cell_coords(const BlockDev& B, long long c, int& i, int& j, int& k) {
  return decode3(c, B.ni, B.nj, B.nk, i, j, k);
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

// Pseudo-node (I, J, K) position: mean centre of the cells
// (I-1+ai, J-1+aj, K-1+ak) with at most one index outside the block.
template <int DIM>
__global__ void __launch_bounds__(256) pseudo_nodes_kernel(ViscArgs a) {
  const BlockDev B = a.blocks[blockIdx.y];
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int I, J, K;
  if (!decode3(n, B.ni + 1, B.nj + 1, DIM == 3 ? B.nk + 1 : 1, I, J, K)) return;
  double acc[DIM];
#pragma unroll
  for (int w = 0; w < DIM; ++w) acc[w] = 0.0;
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
        const double* C = a.centers + B.corigin + p;
#pragma unroll
        for (int c = 0; c < DIM; ++c) acc[c] += C[c * B.vstride];
      }
  const long long nn = node_index(B, I, J, K);
  for (int w = 0; w < DIM; ++w) a.npos[w * B.nnode_total + nn] = acc[w] / (double)cnt;
}

// Green's-theorem gradient of (u.., T) on one face over its dual volume: the
// cell centres CL, CR (values VL, VR) and the face's pseudo-nodes P[m]
// (values W[m]; 2 in 2D, 4 in cyclic order in 3D), vertex values averaged
// along each edge (2D) or over each triangle (3D).  Summed out, the surface
// integral collapses to the closed "diamond" forms evaluated here (D = CR - CL):
//   2D: G = [(V_R - V_L) rot(P1 - P0) + (W0 - W1) rot(D)] / (D x (P1 - P0)),
//       rot(v) = (v_y, -v_x);
//   3D: G = [A (V_R - V_L) - (D x e0)(W0 - W2)/2 - (D x e1)(W1 - W3)/2] / (D . A),
//       e0 = P1 - P3, e1 = P2 - P0, A = e0 x e1 / 2 (D . A is three times the
//       dual volume).
template <int DIM>
__device__ __forceinline__ void dual_gradient(const double* D, const double* VL, const double* VR,
                                              const double (*P)[DIM], const double (*W)[DIM + 1],
                                              double (*G)[DIM]) {
  constexpr int NW = DIM + 1;
  if constexpr (DIM == 2) {
    const double ex = P[1][0] - P[0][0], ey = P[1][1] - P[0][1];
    const double inv = 1.0 / (D[0] * ey - D[1] * ex);
#pragma unroll
    for (int v = 0; v < NW; ++v) {
      const double dv = VR[v] - VL[v], dw = W[0][v] - W[1][v];
      G[v][0] = (dv * ey + dw * D[1]) * inv;
      G[v][1] = (-dv * ex - dw * D[0]) * inv;
    }
  } else {
    double e0[3], e1[3], A[3], b0[3], b1[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) {
      e0[x] = P[1][x] - P[3][x];
      e1[x] = P[2][x] - P[0][x];
    }
    A[0] = 0.5 * (e0[1] * e1[2] - e0[2] * e1[1]);
    A[1] = 0.5 * (e0[2] * e1[0] - e0[0] * e1[2]);
    A[2] = 0.5 * (e0[0] * e1[1] - e0[1] * e1[0]);
    b0[0] = 0.5 * (D[1] * e0[2] - D[2] * e0[1]);
    b0[1] = 0.5 * (D[2] * e0[0] - D[0] * e0[2]);
    b0[2] = 0.5 * (D[0] * e0[1] - D[1] * e0[0]);
    b1[0] = 0.5 * (D[1] * e1[2] - D[2] * e1[1]);
    b1[1] = 0.5 * (D[2] * e1[0] - D[0] * e1[2]);
    b1[2] = 0.5 * (D[0] * e1[1] - D[1] * e1[0]);
    const double inv = 1.0 / (D[0] * A[0] + D[1] * A[1] + D[2] * A[2]);
#pragma unroll
    for (int v = 0; v < NW; ++v) {
      const double dv = VR[v] - VL[v], d02 = W[0][v] - W[2][v], d13 = W[1][v] - W[3][v];
#pragma unroll
      for (int x = 0; x < 3; ++x) G[v][x] = (A[x] * dv - b0[x] * d02 - b1[x] * d13) * inv;
    }
  }
}

// Viscous flux F_v . S (momentum.., energy) from the face gradient G, the face
// velocity uf and the area vector S.
template <int DIM>
__device__ __forceinline__ void viscous_flux(const double (*G)[DIM], const double* uf, const double* S, double mu,
                                             double kcond, double* F) {
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

// Fused 3D pass over a tile of VT_X x VT_Y columns and up to VT_K planes:
// the plane pair (k, k+1) of cells (with a one-cell halo ring) and of
// pseudo-nodes is staged in LDS while the tile marches in k; every face of
// the tile is computed once (x- and y-faces into LDS, the column's k-faces in
// registers) and each cell writes its Rv.
constexpr int VT_X = 16, VT_Y = 16, VT_K = 32;

__global__ void __launch_bounds__(VT_X* VT_Y) viscous_tile_kernel(ViscArgs a) {
  using ML = MetricLayout<3>;
  constexpr int NT = VT_X * VT_Y;
  constexpr int CX = VT_X + 2, CY = VT_Y + 2, NC = CX * CY;  // cells i0-1..i0+VT_X, j0-1..j0+VT_Y
  constexpr int NXn = VT_X + 1, NYn = VT_Y + 1, NN = NXn * NYn;
  constexpr int NFX = NXn * VT_Y, NFY = VT_X * NYn;
  // cell data: 0-2 centre, 3-5 velocity, 6 temperature; node data: velocity, temperature
  __shared__ double sc[2][7][NC];
  __shared__ double sn[2][4][NN];  // pseudo-node values (positions are read from the set-up array)
  __shared__ double fx[4][NFX];
  __shared__ double fy[4][NFY];

  const int tid = threadIdx.x;
  const int tx = tid % VT_X, ty = tid / VT_X;
  const TileDev tile = a.tiles[blockIdx.x];
  const BlockDev B = a.blocks[tile.block];
  const int i0 = tile.i0, j0 = tile.j0, k0 = tile.k0;
  const int k1 = min(k0 + VT_K, B.nk);
  const long long vs = B.vstride;
  const double* met = a.metric + B.morigin;
  const double* cen = a.centers + B.corigin;
  const double* q = a.q + B.origin;
  const int i = i0 + tx, j = j0 + ty;
  const bool own = i < B.ni && j < B.nj;
  const int E = B.ni + 1;                              // node row pitch
  const long long nplane = (long long)(B.nj + 1) * E;  // nodes per plane
  const long long cplane = (long long)B.pj * B.pi;     // padded cells per plane
  // 64-bit parts are per plane (uniform); the in-plane offsets stay 32-bit
  auto node_base = [&](int K) { return node_index(B, i0, j0, K); };
  auto cell_at = [&](int ii, int jj, int kk) { return (long long)kk * cplane + (jj * B.pi + ii); };

  // The next plane's cells are fetched into registers while the current
  // plane's faces are computed (2 items per thread).
  constexpr int HC = (NC + NT - 1) / NT, HN = (NN + NT - 1) / NT;
  double pc[HC][8];  // centre, velocity, rho, p
  bool pv[HC];
  // Along an axis that the block connects to itself end to end, the state of
  // a ghost cell is read from the interior cell it copies (the same values),
  // so the fill between stages can leave those connections out; the ghost
  // cell's centre is still read at the ghost.
  const int wrap = a.wrap ? B.wrap : 0;
  auto wrapc = [](int x, int n, bool on) { return on ? (x < 0 ? x + n : (x >= n ? x - n : x)) : x; };
  // this thread's cell items, the same in every plane of the tile: in-plane
  // offset of the cell and of the cell whose state it holds, how many of i, j
  // lie outside the block, and whether the item is in the staged frame
  int pin[HC], pqin[HC], oxy[HC];
  bool inb[HC];
#pragma unroll
  for (int h = 0; h < HC; ++h) {
    const int e = tid + h * NT;
    const int ii = i0 - 1 + e % CX, jj = j0 - 1 + e / CX;
    oxy[h] = (ii < 0 || ii >= B.ni) + (jj < 0 || jj >= B.nj);
    inb[h] = e < NC && ii <= B.ni && jj <= B.nj;
    pin[h] = jj * B.pi + ii;
    pqin[h] = wrapc(jj, B.nj, wrap & 2) * B.pi + wrapc(ii, B.ni, wrap & 1);
  }
  auto fetch_cells = [&](int kk) {
    const int ko = kk < 0 || kk >= B.nk;
    const long long kp = (long long)kk * cplane, kq = (long long)wrapc(kk, B.nk, wrap & 4) * cplane;
    const long long kc = (long long)min(max(kk, 0), B.nk - 1) * cplane;
#pragma unroll
    for (int h = 0; h < HC; ++h) {
      pv[h] = inb[h] && oxy[h] + ko <= 1;
      // every lane loads (an in-block cell where the item is unused), so no
      // branch join makes the compiler wait for this prefetch early
      const long long p = pv[h] ? kp + pin[h] : kc;
      const long long pq = pv[h] ? kq + pqin[h] : kc;
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        pc[h][x] = cen[x * vs + p];
        pc[h][3 + x] = q[(1 + x) * vs + pq];
      }
      pc[h][6] = q[pq];
      pc[h][7] = q[4 * vs + pq];
    }
  };
  auto store_cells = [&](int slot) {
#pragma unroll
    for (int h = 0; h < HC; ++h) {
      const int e = tid + h * NT;
      if (e >= NC) continue;
#pragma unroll
      for (int w = 0; w < 6; ++w) sc[slot][w][e] = pv[h] ? pc[h][w] : 0.0;
      sc[slot][6][e] = pv[h] ? a.gamma * pc[h][7] / pc[h][6] : 0.0;
    }
  };
  // pseudo-nodes of node plane K from cell planes K-1 (slot sl) and K (slot sh)
  auto make_nodes = [&](int K, int sl, int sh, int slot) {
#pragma unroll
    for (int h = 0; h < HN; ++h) {
      const int e = tid + h * NT;
      const int I = i0 + e % NXn, J = j0 + e / NXn;
      if (e >= NN || I > B.ni || J > B.nj) continue;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      int cnt = 0;
      // cells outside the block in two or more directions were staged as
      // zeros: they add nothing and are not counted
#pragma unroll
      for (int ai = 0; ai < 2; ++ai)
#pragma unroll
        for (int aj = 0; aj < 2; ++aj)
#pragma unroll
          for (int ak = 0; ak < 2; ++ak) {
            const int out = (ai == 0 ? I == 0 : I == B.ni) + (aj == 0 ? J == 0 : J == B.nj) + (ak == 0 ? K == 0 : K == B.nk);
            cnt += out <= 1;
            const int c = (J - j0 + aj) * CX + (I - i0 + ai);  // cell (I-1+ai, J-1+aj) in the halo frame
            const int sls = ak ? sh : sl;
#pragma unroll
            for (int w = 0; w < 4; ++w) acc[w] += sc[sls][3 + w][c];
          }
      // 8 cells, or 6 on an edge of the block, 4 at a corner: the reciprocal
      // from constants (the same bits as 1.0 / cnt, without a division)
      const double rc = cnt == 8 ? 0.125 : (cnt == 6 ? 1.0 / 6.0 : 0.25);
#pragma unroll
      for (int w = 0; w < 4; ++w) sn[slot][w][e] = acc[w] * rc;
    }
  };
  // viscous flux of one face: cells cl (slot sl), cr (slot sr); nodes m0..m3:
  // LDS slot ns, frame index ne (I - i0 + (J - j0) * NXn), global node index go
  auto face = [&](int sl, int cl, int sr, int cr, const int* ns, const int* ne, const long long* go, const double* S,
                  double* F) {
    double D[3], VL[4], VR[4], P[4][3], W[4][4], G[4][3], uf[3];
#pragma unroll
    for (int x = 0; x < 3; ++x) D[x] = sc[sr][x][cr] - sc[sl][x][cl];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      VL[w] = sc[sl][3 + w][cl];
      VR[w] = sc[sr][3 + w][cr];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
      for (int x = 0; x < 3; ++x) P[m][x] = a.npos[x * B.nnode_total + go[m]];
#pragma unroll
      for (int w = 0; w < 4; ++w) W[m][w] = sn[ns[m]][w][ne[m]];
    }
    dual_gradient<3>(D, VL, VR, P, W, G);
#pragma unroll
    for (int x = 0; x < 3; ++x) uf[x] = 0.5 * (VL[x] + VR[x]);
    viscous_flux<3>(G, uf, S, a.mu, a.kcond, F);
  };
  // k-face K of the own column: cells K-1 (slot sl) and K (slot sh), node plane K (slot sn_)
  auto zface = [&](int K, int sl, int sh, int snk, double* F) {
    const int c = (ty + 1) * CX + tx + 1;
    const int n0 = ty * NXn + tx;
    const int ns[4] = {snk, snk, snk, snk};
    const int ne[4] = {n0, n0 + 1, n0 + NXn + 1, n0 + NXn};  // (i,j) (i+1,j) (i+1,j+1) (i,j+1)
    const long long g0 = node_base(K) + (ty * E + tx);
    const long long go[4] = {g0, g0 + 1, g0 + E + 1, g0 + E};
    double S[3];
    const long long p = cell_at(i, j, K);
#pragma unroll
    for (int x = 0; x < 3; ++x) S[x] = met[ML::S(2, x) * vs + p];
    face(sl, c, sh, c, ns, ne, go, S, F);
  };

  // prologue: cell planes k0-1 and k0, node plane k0, the first k-face
  fetch_cells(k0 - 1);
  store_cells(1);
  fetch_cells(k0);
  store_cells(0);
  __syncthreads();
  make_nodes(k0, 1, 0, 0);
  fetch_cells(k0 + 1);
  __syncthreads();
  double fzlo[4] = {0.0, 0.0, 0.0, 0.0};
  if (own) zface(k0, 1, 0, 0, fzlo);

  for (int k = k0; k < k1; ++k) {
    const int s0 = (k - k0) & 1, s1 = s0 ^ 1;  // slots of plane k and k+1
    __syncthreads();  // slot s1 (plane k-1 and node plane k-1) is free
    store_cells(s1);  // plane k+1, fetched during the previous plane
    __syncthreads();
    make_nodes(k + 1, s0, s1, s1);
    __syncthreads();
    const long long nb0 = node_base(k);  // node (i0, j0, k)
    // x-faces (I, j) (flat index e = jr * NXn + I - i0) and y-faces (i, J)
    // (e = (J - j0) * VT_X + i - i0) of plane k
    auto xy_face = [&](bool isx, int e) {
      int I, J;
      if (isx) {
        I = i0 + e % NXn;
        J = j0 + e / NXn;
        if (I > B.ni || J >= B.nj) return;
      } else {
        I = i0 + e % VT_X;
        J = j0 + e / VT_X;
        if (I >= B.ni || J > B.nj) return;
      }
      const int cr = (J - j0 + 1) * CX + (I - i0 + 1);
      const int n0 = (J - j0) * NXn + (I - i0);
      const int ns[4] = {s0, s0, s1, s1};
      // x: (I,j,k) (I,j+1,k) (I,j+1,k+1) (I,j,k+1); y: (i,J,k) (i+1,J,k) (i+1,J,k+1) (i,J,k+1)
      const int n1 = isx ? n0 + NXn : n0 + 1;
      const int ne[4] = {n0, n1, n1, n0};
      const long long g0 = nb0 + ((J - j0) * E + (I - i0));
      const long long g1 = isx ? g0 + E : g0 + 1;
      const long long go[4] = {g0, g1, g1 + nplane, g0 + nplane};
      double S[3], F[4];
      const long long p = cell_at(I, J, k);
#pragma unroll
      for (int x = 0; x < 3; ++x) S[x] = met[ML::S(isx ? 0 : 1, x) * vs + p];
      face(s0, isx ? cr - 1 : cr - CX, s0, cr, ns, ne, go, S, F);
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        if (isx)
          fx[w][e] = F[w];
        else
          fy[w][e] = F[w];
      }
    };
    // first NT of each kind, then the remaining NFX - NT x-faces and NFY - NT
    // y-faces in one shared round (on one wave instead of two rounds)
    static_assert(NFX - NT + NFY - NT <= 64, "leftover faces fit one wavefront");
    // (unrolled, so the two faces' loads and arithmetic interleave: 231 VGPRs,
    // still the two waves per SIMD that the LDS allows; 1.18 -> 1.13 ms on 256^3)
#pragma unroll
    for (int r = 0; r < 2; ++r) xy_face(r == 0, tid);
    if (tid < NFX - NT + NFY - NT) {
      const bool isx = tid < NFX - NT;
      xy_face(isx, NT + (isx ? tid : tid - (NFX - NT)));
    }
    double fzhi[4];
    if (own) zface(k + 1, s0, s1, s1, fzhi);
    // the cell's inverse volume, then plane k+2 while the divergence and the
    // next plane's staging run (issued after every load the rest of this
    // plane waits for, so no wait covers the prefetch)
    const double ivc = met[ML::INVVOL * vs + cell_at(min(i, B.ni - 1), min(j, B.nj - 1), k)];
    // (unconditional: after the tile's last plane this reads plane k1 + 1 <=
    // nk + 1, inside the padded block, and the values go unused)
    fetch_cells(k + 2);
    __syncthreads();
    if (own) {
      const double iv = ivc;
      const long long cell = B.packed + ((long long)k * B.nj + j) * B.ni + i;
      const int ex = ty * NXn + tx, ey = ty * VT_X + tx;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const double acc = (fx[w][ex + 1] - fx[w][ex]) + (fy[w][ey + VT_X] - fy[w][ey]) + (fzhi[w] - fzlo[w]);
        a.rv[w * B.ncell_total + cell] = acc * iv;
        fzlo[w] = fzhi[w];
      }
    }
  }
}

// Fused 2D pass over a VT2 x VT2 tile: cells with a one-cell halo ring
// (centre, velocity, temperature) and the tile's pseudo-node values in LDS,
// every face once (own low faces plus the tile's high edges), Rv per cell.
// Same arithmetic as the per-face 2D kernels.
constexpr int VT2 = 16;

__global__ void __launch_bounds__(VT2* VT2) viscous_tile2d_kernel(ViscArgs a) {
  using ML = MetricLayout<2>;
  constexpr int NT = VT2 * VT2;
  constexpr int CX = VT2 + 2, NC = CX * CX;
  constexpr int NXn = VT2 + 1, NN = NXn * NXn;
  constexpr int NFX = NXn * VT2, NFY = VT2 * NXn;
  __shared__ double sc[5][NC];  // centre x, y, velocity u, v, temperature
  __shared__ double sn[3][NN];  // pseudo-node u, v, T
  __shared__ double fx[3][NFX];
  __shared__ double fy[3][NFY];

  const int tid = threadIdx.x;
  const int tx = tid % VT2, ty = tid / VT2;
  const TileDev tile = a.tiles[blockIdx.x];
  const BlockDev B = a.blocks[tile.block];
  const int i0 = tile.i0, j0 = tile.j0;
  const long long vs = B.vstride;
  const double* met = a.metric + B.morigin;
  const double* cen = a.centers + B.corigin;
  const double* q = a.q + B.origin;
  const int E = B.ni + 1;
  const long long nb0 = node_index(B, i0, j0, 0);
  // (periodic neighbours' state through the wrap, as in the 3D pass)
  const int wrap = a.wrap ? B.wrap : 0;
  auto wrapc = [](int x, int n, bool on) { return on ? (x < 0 ? x + n : (x >= n ? x - n : x)) : x; };

  for (int e = tid; e < NC; e += NT) {
    const int ii = i0 - 1 + e % CX, jj = j0 - 1 + e / CX;
    const int out = (ii < 0 || ii >= B.ni) + (jj < 0 || jj >= B.nj);
    if (ii <= B.ni && jj <= B.nj && out <= 1) {
      const long long p = jj * B.pi + ii;
      const long long pq = (long long)wrapc(jj, B.nj, wrap & 2) * B.pi + wrapc(ii, B.ni, wrap & 1);
      sc[0][e] = cen[p];
      sc[1][e] = cen[vs + p];
      sc[2][e] = q[vs + pq];
      sc[3][e] = q[2 * vs + pq];
      sc[4][e] = a.gamma * q[3 * vs + pq] / q[pq];
    } else {
#pragma unroll
      for (int w = 0; w < 5; ++w) sc[w][e] = 0.0;
    }
  }
  __syncthreads();
  for (int e = tid; e < NN; e += NT) {
    const int I = i0 + e % NXn, J = j0 + e / NXn;
    if (I > B.ni || J > B.nj) continue;
    double acc[3] = {0.0, 0.0, 0.0};
    int cnt = 0;
    // corner cells (outside in both directions) were staged as zeros: they
    // add nothing and are not counted
#pragma unroll
    for (int ai = 0; ai < 2; ++ai)
#pragma unroll
      for (int aj = 0; aj < 2; ++aj) {
        const int out = (ai == 0 ? I == 0 : I == B.ni) + (aj == 0 ? J == 0 : J == B.nj);
        cnt += out <= 1;
        const int c = (J - j0 + aj) * CX + (I - i0 + ai);
#pragma unroll
        for (int w = 0; w < 3; ++w) acc[w] += sc[2 + w][c];
      }
    // 4 cells, 3 at a corner of the block (the same bits as 1.0 / cnt)
    const double rc = cnt == 4 ? 0.25 : 1.0 / 3.0;
#pragma unroll
    for (int w = 0; w < 3; ++w) sn[w][e] = acc[w] * rc;
  }
  __syncthreads();
  // face between LDS cells cl and cr; pseudo-nodes n0, n1 (frame) / g0, g1 (global)
  auto face = [&](int cl, int cr, int n0, int n1, long long g0, long long g1, const double* S, double* F) {
    double D[2], VL[3], VR[3], P[2][2], W[2][3], G[3][2], uf[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) D[x] = sc[x][cr] - sc[x][cl];
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      VL[w] = sc[2 + w][cl];
      VR[w] = sc[2 + w][cr];
      W[0][w] = sn[w][n0];
      W[1][w] = sn[w][n1];
    }
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      P[0][x] = a.npos[x * B.nnode_total + g0];
      P[1][x] = a.npos[x * B.nnode_total + g1];
    }
    dual_gradient<2>(D, VL, VR, P, W, G);
#pragma unroll
    for (int x = 0; x < 2; ++x) uf[x] = 0.5 * (VL[x] + VR[x]);
    viscous_flux<2>(G, uf, S, a.mu, a.kcond, F);
  };
  auto xface = [&](int I, int jj, double* F) {  // nodes (I, j), (I, j+1)
    const int cr = (jj - j0 + 1) * CX + (I - i0 + 1);
    const int n0 = (jj - j0) * NXn + (I - i0);
    const long long g0 = nb0 + ((jj - j0) * E + (I - i0));
    double S[2];
    const long long p = jj * B.pi + I;
    S[0] = met[ML::S(0, 0) * vs + p];
    S[1] = met[ML::S(0, 1) * vs + p];
    face(cr - 1, cr, n0, n0 + NXn, g0, g0 + E, S, F);
  };
  auto yface = [&](int ii, int J, double* F) {  // nodes (i, J), (i+1, J)
    const int cr = (J - j0 + 1) * CX + (ii - i0 + 1);
    const int n0 = (J - j0) * NXn + (ii - i0);
    const long long g0 = nb0 + ((J - j0) * E + (ii - i0));
    double S[2];
    const long long p = J * B.pi + ii;
    S[0] = met[ML::S(1, 0) * vs + p];
    S[1] = met[ML::S(1, 1) * vs + p];
    face(cr - CX, cr, n0, n0 + 1, g0, g0 + 1, S, F);
  };
  const int i = i0 + tx, j = j0 + ty;
  if (i <= B.ni && j < B.nj) {
    double F[3];
    xface(i, j, F);
#pragma unroll
    for (int w = 0; w < 3; ++w) fx[w][ty * NXn + tx] = F[w];
  }
  if (i < B.ni && j <= B.nj) {
    double F[3];
    yface(i, j, F);
#pragma unroll
    for (int w = 0; w < 3; ++w) fy[w][ty * VT2 + tx] = F[w];
  }
  if (tid < VT2) {  // x-faces of the tile's high i-edge
    const int I = i0 + VT2, jj = j0 + tid;
    if (I <= B.ni && jj < B.nj) {
      double F[3];
      xface(I, jj, F);
#pragma unroll
      for (int w = 0; w < 3; ++w) fx[w][tid * NXn + VT2] = F[w];
    }
  } else if (tid < 2 * VT2) {  // y-faces of the tile's high j-edge
    const int ii = i0 + tid - VT2, J = j0 + VT2;
    if (ii < B.ni && J <= B.nj) {
      double F[3];
      yface(ii, J, F);
#pragma unroll
      for (int w = 0; w < 3; ++w) fy[w][VT2 * VT2 + tid - VT2] = F[w];
    }
  }
  __syncthreads();
  if (i < B.ni && j < B.nj) {
    const long long p = j * B.pi + i;
    const double iv = met[ML::INVVOL * vs + p];
    const long long cell = B.packed + (long long)j * B.ni + i;
    const int ex = ty * NXn + tx, ey = ty * VT2 + tx;
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const double acc = (fx[w][ex + 1] - fx[w][ex]) + (fy[w][ey + VT2] - fy[w][ey]);
      a.rv[w * B.ncell_total + cell] = acc * iv;
    }
  }
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

hipError_t launch_pseudo_nodes(int dim, const ViscArgs& a, long long max_nodes, int nblocks, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(pseudo_nodes_kernel<2>, grid_of(max_nodes, nblocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(pseudo_nodes_kernel<3>, grid_of(max_nodes, nblocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

void viscous_tile_shape(int dim, int* tx, int* ty, int* tk) {
  *tx = dim == 2 ? VT2 : VT_X;
  *ty = dim == 2 ? VT2 : VT_Y;
  *tk = dim == 2 ? 1 : VT_K;
}

hipError_t launch_viscous(int dim, const ViscArgs& a, hipStream_t s) {
  if (a.ntiles <= 0) return hipSuccess;
  if (dim == 2)
    hipLaunchKernelGGL(viscous_tile2d_kernel, dim3(a.ntiles), dim3(VT2 * VT2), 0, s, a);
  else
    hipLaunchKernelGGL(viscous_tile_kernel, dim3(a.ntiles), dim3(VT_X * VT_Y), 0, s, a);
  return hipGetLastError();
}

}  // namespace cfd
