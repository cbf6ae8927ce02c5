"""MI355X-native FP64 hot path of a structured multi-block Euler solver
(arXiv 2012.02925): HIP kernels behind the C ABI of libcfdhip.so.

Submodules:
  capi    ctypes binding of the C entry points (same names)
  solver  Solver: owns a context, its workspace tensor and the marshalling
  build   builds libcfdhip.so in-tree with hipcc for gfx950
"""
__all__ = ["capi", "solver", "build"]
