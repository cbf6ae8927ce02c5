// Host-side launch templates of the stage kernel: one instantiation per
// dimension, limiter, tile shape, face flux and farfield flag.  The 2D and 3D
// instantiations live in separate translation units (stage2d.hip,
// stage3d.hip) so they compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "stage_kernel.h"

namespace cfd {

template <int DIM, int LIM, int TX, int TY, int KC, int FLUX>
inline hipError_t launch_stage_t(bool ff, const StageArgs& a, int grid, bool persistent, hipStream_t s) {
  if (grid <= 0) return hipSuccess;
  void (*k)(StageArgs) = ff ? (a.dtmin ? stage_kernel<DIM, LIM, TX, TY, KC, FLUX, true, true>
                                       : stage_kernel<DIM, LIM, TX, TY, KC, FLUX, true, false>)
                            : (a.dtmin ? stage_kernel<DIM, LIM, TX, TY, KC, FLUX, false, true>
                                       : stage_kernel<DIM, LIM, TX, TY, KC, FLUX, false, false>);
  if (persistent) {
    // persistent launch: as many workgroups as can be resident at once on
    // the device (compute units x workgroups per unit for this kernel), each
    // walking the tile list with the kernel's grid-stride loop.  Cached per
    // kernel (one device type per process).
    static int resident[4] = {0, 0, 0, 0};
    const int slot = (ff ? 2 : 0) + (a.dtmin ? 1 : 0);
    if (resident[slot] == 0) {
      int dev = 0, ncu = 0, per = 0;
      hipError_t e = hipGetDevice(&dev);
      if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
      if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, TX * TY, 0);
      if (e != hipSuccess) return e;
      resident[slot] = ncu * per > 0 ? ncu * per : 1;
    }
    grid = grid < resident[slot] ? grid : resident[slot];
  }
  hipLaunchKernelGGL(k, dim3(grid), dim3(TX * TY), 0, s, a);
  return hipGetLastError();
}

template <int DIM, int TX, int TY, int KC, int FLUX>
inline hipError_t launch_stage_lim(int lim, bool ff, const StageArgs& a, int grid, bool pers, hipStream_t s) {
  switch (lim) {
    case LIM_NONE: return launch_stage_t<DIM, LIM_NONE, TX, TY, KC, FLUX>(ff, a, grid, pers, s);
    case LIM_VANLEER: return launch_stage_t<DIM, LIM_VANLEER, TX, TY, KC, FLUX>(ff, a, grid, pers, s);
    case LIM_FROZEN: return launch_stage_t<DIM, LIM_FROZEN, TX, TY, KC, FLUX>(ff, a, grid, pers, s);
    case LIM_VANALBADA0: return launch_stage_t<DIM, LIM_VANALBADA0, TX, TY, KC, FLUX>(ff, a, grid, pers, s);
    default: return launch_stage_t<DIM, LIM_VANALBADA, TX, TY, KC, FLUX>(ff, a, grid, pers, s);
  }
}

template <int DIM, int TX, int TY, int KC>
inline hipError_t launch_stage_flux(int flux, int lim, bool ff, const StageArgs& a, int grid, bool pers,
                                    hipStream_t s) {
  switch (flux) {
    case FLUX_VANLEER_FVS: return launch_stage_lim<DIM, TX, TY, KC, FLUX_VANLEER_FVS>(lim, ff, a, grid, pers, s);
    case FLUX_STEGER_WARMING:
      return launch_stage_lim<DIM, TX, TY, KC, FLUX_STEGER_WARMING>(lim, ff, a, grid, pers, s);
    default: return launch_stage_lim<DIM, TX, TY, KC, FLUX_ROE>(lim, ff, a, grid, pers, s);
  }
}

hipError_t launch_stage_2d(int flux, int lim, int variant, bool ff, const StageArgs& a, int grid, bool pers,
                           hipStream_t s);
hipError_t launch_stage_3d(int flux, int lim, int variant, bool ff, const StageArgs& a, int grid, bool pers,
                           hipStream_t s);
hipError_t launch_stage_3d_fvs(int flux, int lim, int variant, bool ff, const StageArgs& a, int grid, bool pers,
                               hipStream_t s);

}  // namespace cfd
