// Device-visible tables and indexing shared by the host planner and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cfd {

constexpr int NG = 2;    // ghost layers: the four-cell MUSCL stencil of eq. (flux)
constexpr int MAXV = 5;  // variables in 3D
constexpr int FARFIELD_MASK_SHIFT = 1 << 8;  // BlockDev::wall_mask: farfield bits above the wall bits
// The CFL time step's minimum of Omega/lambda is reduced into DT_SLOTS slots
// (workgroup w into slot w mod DT_SLOTS, one atomic each) so that thousands
// of workgroups do not all update one address; the promote kernel takes the
// minimum over the slots (an exact minimum, whatever the order).
constexpr int DT_SLOTS = 64;

// One structured block in the workspace.  Every padded array of the block
// (state variables, metric components) shares the same geometry:
// element (i, j, k) with i in [-2, ni+2), j in [-2, nj+2), k in [-2, nk+2)
// (k = 0 only in 2D) lives at  origin + (k * pj + j) * pi + i  of its array,
// and consecutive arrays are vstride doubles apart.  origin is 16-double
// aligned so every interior row starts on a 128-byte boundary.
struct BlockDev {
  int ni, nj, nk;
  int pi, pj;              // row pitch (doubles), rows per k-plane
  int wall_mask;           // bit f: face f carries a slip-wall patch; bit f + 8: a farfield patch
  int wrap;                // bit d: axis d is connected to itself end to end (periodic, no reorientation)
  long long vstride;       // doubles between two padded arrays of this block
  long long origin;        // offset of interior (0,0,0) of array 0 within a state buffer
  long long morigin;       // offset of interior (0,0,0) of metric array 0 within the metric buffer
  long long forigin;       // offset of interior (0,0,0) of face-scratch array 0 (adjoint)
  long long lorigin;       // offset of interior (0,0,0) of frozen-limiter array 0 (d * nvar + v)
  long long corigin;       // offset of interior (0,0,0) of cell-centre array 0 (viscous)
  long long packed;        // first cell of the block in the packed [var][cell] layout
  long long node0;         // first node of the block in the concatenated node layout
  long long ncell_total;   // cells of all blocks (stride between packed variables)
  long long nnode_total;   // nodes of all blocks (stride between node coordinates)
};

__host__ __device__ inline long long pidx(const BlockDev& b, int i, int j, int k) {
  return ((long long)k * b.pj + j) * (long long)b.pi + i;
}

// Metric arrays of a block: for direction d and component c the face area
// vector S^d_c of the low face of cell (i,j,k) is array d*DIM + c; the
// reciprocal cell volume is array DIM*DIM.
template <int DIM>
struct MetricLayout {
  static constexpr int S(int d, int c) { return d * DIM + c; }
  static constexpr int INVVOL = DIM * DIM;
  static constexpr int COUNT = DIM * DIM + 1;
};

// One direction of a connection: the donor's first two interior layers at
// its face range fill the receiver's two ghost layers at its range.
// Exchange-buffer segment layout: [var][t2][t1][layer] (layer 0 = adjacent).
struct TransferDev {
  int rblock, rface, dblock, dface;
  int rlo0, rlo1, len0, len1;      // receiver range (len1 = 1 in 2D)
  int dlo0, dlo1, dlen0, dlen1;    // donor range
  int orient;                      // receiver offset -> donor offset map
  int pad_;
  long long buf;                   // offset of the segment in the exchange buffer
};

enum PatchKind {
  PK_SLIP_WALL = 1,
  PK_SUP_INFLOW = 2,
  PK_EXTRAP_OUTFLOW = 3,
  PK_FARFIELD = 4,
  PK_SUB_INFLOW = 5,
  PK_SUB_OUTFLOW = 6,
  PK_NOSLIP_WALL = 7
};

struct PatchDev {
  int block, face, kind, param;    // param: slot of the patch's parameters (MAXV doubles each), or -1
  int lo0, lo1, len0, len1;
};

// A work chunk of a ghost-fill launch: CHUNK consecutive elements of one item.
// kind 0: pack a transfer; 1: fill a physical patch; 2: unpack a transfer;
// 3: copy a transfer from donor interior to receiver ghosts directly.
struct ChunkDev {
  int kind, item, start, count;
};
constexpr int CHUNK = 256;

struct TileDev {
  int block, i0, j0, k0;
};

// Maps a receiver tangential offset (r1, r2) to the donor offset.
__host__ __device__ inline void orient_map(int orient, int r1, int r2, int dlen0, int dlen1, int& d1, int& d2) {
  int s1 = (orient & 4) ? r2 : r1;
  int s2 = (orient & 4) ? r1 : r2;
  d1 = (orient & 1) ? (dlen0 - 1 - s1) : s1;
  d2 = (orient & 2) ? (dlen1 - 1 - s2) : s2;
}

// Cell (i,j,k) of layer `layer` of a face (0 = adjacent to the face, counted
// inward for interior layers; ghost = true counts outward, layer 0 = first
// ghost layer) at tangential cell coordinates (t1, t2).
__host__ __device__ inline void face_cell(const BlockDev& b, int dim, int face, int layer, bool ghost,
                                          int t1, int t2, int& i, int& j, int& k) {
  int axis = face >> 1;
  bool hi = face & 1;
  int n = axis == 0 ? b.ni : (axis == 1 ? b.nj : b.nk);
  int nrm;
  if (ghost)
    nrm = hi ? n + layer : -1 - layer;
  else
    nrm = hi ? n - 1 - layer : layer;
  // tangential axes in increasing order
  int ta = axis == 0 ? 1 : 0;
  int tb = axis == 2 ? 1 : 2;
  int c[3] = {0, 0, 0};
  c[axis] = nrm;
  c[ta] = t1;
  if (dim == 3) c[tb] = t2;
  i = c[0];
  j = c[1];
  k = c[2];
}

}  // namespace cfd
