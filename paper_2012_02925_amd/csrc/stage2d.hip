// 2D stage-kernel instantiations (tile variants of stage_variants(2)).
#include "stage_launch.h"

namespace cfd {

hipError_t launch_stage_2d(int flux, int lim, int variant, bool ff, const StageArgs& a, int grid, bool pers,
                           hipStream_t s) {
  switch (variant) {
    case 0: return launch_stage_flux<2, 64, 4, 1>(flux, lim, ff, a, grid, pers, s);
    case 1: return launch_stage_flux<2, 32, 8, 1>(flux, lim, ff, a, grid, pers, s);
    default: return launch_stage_flux<2, 16, 16, 1>(flux, lim, ff, a, grid, pers, s);
  }
}

}  // namespace cfd
