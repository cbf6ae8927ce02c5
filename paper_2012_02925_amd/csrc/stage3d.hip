// 3D stage-kernel instantiations (tile variants of stage_variants(3)).  The
// Roe kernels and the flux-vector-splitting kernels are separate translation
// units so they compile in parallel.
#include "stage_launch.h"

namespace cfd {

#ifdef CFD_STAGE3D_FVS
hipError_t launch_stage_3d_fvs(int flux, int lim, int variant, bool ff, const StageArgs& a, int grid, bool pers,
                               hipStream_t s) {
  switch (variant) {
    case 0: return launch_stage_flux<3, 64, 4, 32>(flux, lim, ff, a, grid, pers, s);
    case 1: return launch_stage_flux<3, 32, 8, 32>(flux, lim, ff, a, grid, pers, s);
    default: return launch_stage_flux<3, 32, 8, 64>(flux, lim, ff, a, grid, pers, s);
  }
}
#else
hipError_t launch_stage_3d(int flux, int lim, int variant, bool ff, const StageArgs& a, int grid, bool pers,
                           hipStream_t s) {
  if (flux != FLUX_ROE) return launch_stage_3d_fvs(flux, lim, variant, ff, a, grid, pers, s);
  switch (variant) {
    case 0: return launch_stage_lim<3, 64, 4, 32, FLUX_ROE>(lim, ff, a, grid, pers, s);
    case 1: return launch_stage_lim<3, 32, 8, 32, FLUX_ROE>(lim, ff, a, grid, pers, s);
    default: return launch_stage_lim<3, 32, 8, 64, FLUX_ROE>(lim, ff, a, grid, pers, s);
  }
}
#endif

}  // namespace cfd
