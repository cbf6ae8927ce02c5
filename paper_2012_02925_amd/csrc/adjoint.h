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
  double* out;              // packed: out = scale * Qbar (nullable)
  double* acc;              // packed: acc += scale * Qbar (nullable)
  double scale;
  Gas gas;
  double half_eps, kappa, efix, half_inv_efix;
  double e2[MAXV];
};

hipError_t launch_vjp_face(int dim, int lim, const VjpArgs& a, long long max_faces, int nb, hipStream_t s);
hipError_t launch_vjp_cell(int dim, int lim, const VjpArgs& a, long long max_padded, int nb, hipStream_t s);
hipError_t launch_vjp_ghost(int dim, const VjpArgs& a, const ChunkDev* chunks, int begin, int count, hipStream_t s);
hipError_t launch_vjp_finalize(int dim, const VjpArgs& a, long long max_cells, int nb, hipStream_t s);
hipError_t launch_vjp_inflow_reduce(int dim, const VjpArgs& a, const int* inflow_patches, int n, hipStream_t s);
hipError_t launch_objective(int dim, const VjpArgs& a, const ChunkDev* chunks, int begin, int count, hipStream_t s);
hipError_t launch_objective_sum(const VjpArgs& a, const int* wall_patches, int nwall, double* J, hipStream_t s);
hipError_t launch_node_vjp_2d(const VjpArgs& a, double* Xb, long long max_nodes, int nb, hipStream_t s);
hipError_t launch_uniform_state_vjp(int dim, const double* Qbar, long long ncells, double* partial, int nparts,
                                    double* thetabar, Gas g, const double* theta, hipStream_t s);

}  // namespace cfd
