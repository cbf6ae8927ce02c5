// Launch interface of the adjoint (residual VJP) kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "cfd_internal.h"
#include "device_math.h"

namespace cfd {

struct VjpArgs {
  const BlockDev* blocks;
  const TransferDev* xfers;
  const PatchDev* patches;
  int npatches;
  const double* q;          // state the residual is taken at (primitive, padded, ghosts filled)
  const double* metric;
  const double* nodes;
  const double* Rb;         // packed residual cotangent
  double* facebar;          // per-face scratch: [dir][qL-bar(nv), qR-bar(nv), pw-bar, cL, cR]
  double* qbar;             // primitive cotangent, padded state layout
  double* metricbar;        // accumulated dJ/dS (metric slots) and dJ/dOmega (volume slot)
  double* thetabar;         // accumulated dJ/d(inflow state), MAXV per inflow patch
  double* inflow_part;      // per-patch partial sums
  const long long* part_offset;  // offset of each patch's partials
  const int* facemap;       // per block face and tangential position: transfer (>= 0, as donor) or -(patch+1)
  const long long* fmap_off;  // offset of block b, face f in facemap: fmap_off[b * 6 + f]
  const TileDev* vtiles;    // 2D tiles of the fused face/cell pass
  const int* inflow_list;   // inflow patch ids in reduction order
  int ninflow;
  double* out;              // packed: out = scale * Qbar (nullable)
  double* acc;              // packed accumulator (nullable), see acc_mode
  int acc_mode;             // acc += (bit 0: scale * Qbar) + (bit 1: Rb)
  int tile_bc;              // 2D: the tile pass finalizes cells next to physical patches
  double scale;
  Gas gas;
  double half_eps, kappa, efix, half_inv_efix;
  double e2[MAXV];
};

hipError_t launch_vjp_face(int dim, int lim, const VjpArgs& a, long long max_faces, int nb, hipStream_t s);
hipError_t launch_vjp_cell(int dim, int lim, const VjpArgs& a, long long max_padded, int nb, hipStream_t s);
// tile edge of the fused 2D pass
constexpr int VJP_TILE = 16;
constexpr int FMAP_NONE = -2147483647 - 1;
hipError_t launch_vjp_tile2d(int lim, const VjpArgs& a, int ntiles, hipStream_t s);
hipError_t launch_vjp_boundary_gather(int dim, const VjpArgs& a, long long max_face_area, int nb, hipStream_t s);
hipError_t launch_vjp_inflow_reduce(int dim, const VjpArgs& a, hipStream_t s);
hipError_t launch_vjp_finalize(int dim, const VjpArgs& a, long long max_cells, int nb, hipStream_t s);
hipError_t launch_objective(int dim, const VjpArgs& a, const ChunkDev* chunks, int begin, int count, hipStream_t s);
hipError_t launch_objective_sum(const VjpArgs& a, const int* wall_patches, int nwall, double* J, hipStream_t s);
hipError_t launch_node_vjp(int dim, const VjpArgs& a, double* Xb, long long max_nodes, int nb, hipStream_t s);
hipError_t launch_uniform_state_vjp(int dim, const double* Qbar, long long ncells, double* partial, int nparts,
                                    double* thetabar, Gas g, const double* theta, hipStream_t s);

}  // namespace cfd
