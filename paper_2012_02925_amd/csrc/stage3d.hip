// 3D stage-kernel instantiations (tile variants of stage_variants(3)).
#include "stage_launch.h"

namespace cfd {

hipError_t launch_stage_3d(int flux, int lim, int variant, bool ff, const StageArgs& a, int grid, hipStream_t s) {
  switch (variant) {
    case 0: return launch_stage_flux<3, 64, 4, 32>(flux, lim, ff, a, grid, s);
    case 1: return launch_stage_flux<3, 32, 8, 32>(flux, lim, ff, a, grid, s);
    default: return launch_stage_flux<3, 32, 8, 64>(flux, lim, ff, a, grid, s);
  }
}

}  // namespace cfd
