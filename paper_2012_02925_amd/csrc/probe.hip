// Streaming-bandwidth probe: a plain kernel with the stage kernel's memory
// traffic per cell and none of its arithmetic, so the attainable HBM rate for
// that read:write mix can be measured on the same GPU (the practical ceiling
// the stage kernel's bandwidth is compared with).
//
// Per element e of n: reads element e of R arrays, writes element e of W
// arrays (the sum of the reads), each array n doubles, structure of arrays,
// one double per lane per array (the stage kernel's 8-byte coalesced loads)
// or, with VEC = 2, two consecutive elements per lane (16-byte loads).
#include <hip/hip_runtime.h>

#include "../../include/cfdhip.h"

namespace {

template <int R, int W, int VEC>
__global__ void __launch_bounds__(256) stream_kernel(const double* __restrict__ src, double* __restrict__ dst,
                                                     long long n) {
  const long long nv = n / VEC;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < nv; e += stride) {
    if constexpr (VEC == 1) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < R; ++a) s += src[a * n + e];
#pragma unroll
      for (int b = 0; b < W; ++b) dst[b * n + e] = s + (double)b;
    } else {
      double2 s = make_double2(0.0, 0.0);
#pragma unroll
      for (int a = 0; a < R; ++a) {
        const double2 x = reinterpret_cast<const double2*>(src + a * n)[e];
        s.x += x.x;
        s.y += x.y;
      }
#pragma unroll
      for (int b = 0; b < W; ++b) reinterpret_cast<double2*>(dst + b * n)[e] = make_double2(s.x + b, s.y + b);
    }
  }
}

template <int R, int W>
hipError_t launch(int vec, int grid, const double* src, double* dst, long long n, hipStream_t s) {
  if (vec == 2)
    hipLaunchKernelGGL((stream_kernel<R, W, 2>), dim3(grid), dim3(256), 0, s, src, dst, n);
  else
    hipLaunchKernelGGL((stream_kernel<R, W, 1>), dim3(grid), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

}  // namespace

extern "C" cfd_status cfd_stream_probe(int reads, int writes, int vec, const double* dev_src, double* dev_dst,
                                       long long n, int reps, void* hip_stream, double* ms_out) {
  if (!dev_src || !dev_dst || !ms_out || n <= 0 || reps <= 0 || (vec != 1 && vec != 2) || (n % vec) != 0)
    return CFD_ERR_ARG;
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const long long items = n / vec;
  const int grid = (int)((items + 255) / 256 < 1048576 ? (items + 255) / 256 : 1048576);
  auto go = [&]() -> hipError_t {
    if (reads == 4 && writes == 1) return launch<4, 1>(vec, grid, dev_src, dev_dst, n, s);
    if (reads == 3 && writes == 1) return launch<3, 1>(vec, grid, dev_src, dev_dst, n, s);
    if (reads == 20 && writes == 5) return launch<20, 5>(vec, grid, dev_src, dev_dst, n, s);
    if (reads == 15 && writes == 5) return launch<15, 5>(vec, grid, dev_src, dev_dst, n, s);
    if (reads == 1 && writes == 1) return launch<1, 1>(vec, grid, dev_src, dev_dst, n, s);
    return hipErrorInvalidValue;
  };
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return CFD_ERR_HIP;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return CFD_ERR_HIP;
  }
  cfd_status st = CFD_OK;
  if (go() != hipSuccess) st = CFD_ERR_ARG;  // unsupported (reads, writes) pair, or launch failure
  if (st == CFD_OK && hipEventRecord(e0, s) != hipSuccess) st = CFD_ERR_HIP;
  for (int r = 0; r < reps && st == CFD_OK; ++r)
    if (go() != hipSuccess) st = CFD_ERR_HIP;
  if (st == CFD_OK && hipEventRecord(e1, s) != hipSuccess) st = CFD_ERR_HIP;
  float ms = 0.0f;
  if (st == CFD_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    st = CFD_ERR_HIP;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == CFD_OK) *ms_out = (double)ms / reps;
  return st;
}
