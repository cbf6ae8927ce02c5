// 3D stage kernels with the flux-vector splittings (see stage3d.hip).
#define CFD_STAGE3D_FVS
#include "stage3d.hip"
