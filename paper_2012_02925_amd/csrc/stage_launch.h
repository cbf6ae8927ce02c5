// Host-side launch templates of the stage kernel: one instantiation per
// dimension, limiter, tile shape, face flux and farfield flag.  The 2D and 3D
// instantiations live in separate translation units (stage2d.hip,
// stage3d.hip) so they compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "stage_kernel.h"

namespace cfd {

template <int DIM, int LIM, int TX, int TY, int KC, int FLUX>
inline hipError_t launch_stage_t(bool ff, const StageArgs& a, int grid, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  const dim3 g(grid), b(TX * TY);
  if (ff) {
    if (a.dtmin)
      hipLaunchKernelGGL((stage_kernel<DIM, LIM, TX, TY, KC, FLUX, true, true>), g, b, 0, s, a);
    else
      hipLaunchKernelGGL((stage_kernel<DIM, LIM, TX, TY, KC, FLUX, true, false>), g, b, 0, s, a);
  } else {
    if (a.dtmin)
      hipLaunchKernelGGL((stage_kernel<DIM, LIM, TX, TY, KC, FLUX, false, true>), g, b, 0, s, a);
    else
      hipLaunchKernelGGL((stage_kernel<DIM, LIM, TX, TY, KC, FLUX, false, false>), g, b, 0, s, a);
  }
  return hipGetLastError();
}

template <int DIM, int TX, int TY, int KC, int FLUX>
inline hipError_t launch_stage_lim(int lim, bool ff, const StageArgs& a, int grid, hipStream_t s) {
  switch (lim) {
    case LIM_NONE: return launch_stage_t<DIM, LIM_NONE, TX, TY, KC, FLUX>(ff, a, grid, s);
    case LIM_VANLEER: return launch_stage_t<DIM, LIM_VANLEER, TX, TY, KC, FLUX>(ff, a, grid, s);
    case LIM_FROZEN: return launch_stage_t<DIM, LIM_FROZEN, TX, TY, KC, FLUX>(ff, a, grid, s);
    default: return launch_stage_t<DIM, LIM_VANALBADA, TX, TY, KC, FLUX>(ff, a, grid, s);
  }
}

template <int DIM, int TX, int TY, int KC>
inline hipError_t launch_stage_flux(int flux, int lim, bool ff, const StageArgs& a, int grid, hipStream_t s) {
  switch (flux) {
    case FLUX_VANLEER_FVS: return launch_stage_lim<DIM, TX, TY, KC, FLUX_VANLEER_FVS>(lim, ff, a, grid, s);
    case FLUX_STEGER_WARMING: return launch_stage_lim<DIM, TX, TY, KC, FLUX_STEGER_WARMING>(lim, ff, a, grid, s);
    default: return launch_stage_lim<DIM, TX, TY, KC, FLUX_ROE>(lim, ff, a, grid, s);
  }
}

hipError_t launch_stage_2d(int flux, int lim, int variant, bool ff, const StageArgs& a, int grid, hipStream_t s);
hipError_t launch_stage_3d(int flux, int lim, int variant, bool ff, const StageArgs& a, int grid, hipStream_t s);
hipError_t launch_stage_3d_fvs(int flux, int lim, int variant, bool ff, const StageArgs& a, int grid,
                               hipStream_t s);

}  // namespace cfd
