"""CPU FP64 oracle for the structured-grid Euler hot path.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP path is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does
and must fail loudly when its own compiled library is missing.

It is written from the paper (Xue, Jackson, Roy, arXiv 2012.02925) with plain
PyTorch CPU tensor operations in float64: no blocking, fusion or reordering
beyond what the formulas state.  It shares no code with the HIP library; both
take their inputs from the neutral ``synth`` package.

Modules
-------
gas      conserved/primitive variables and the inviscid normal flux (Sec. 2, eq. 2)
metrics  face area vectors and cell volumes from the nodes (Sec. 2, finite-volume form)
muscl    limiter functions and the kappa-form MUSCL face states (Sec. 7.2 V4, eq. (flux))
roe      Roe flux-difference splitting (Sec. 2, cited Roe 1981)
ghosts   connected-boundary and physical-boundary ghost fill (Sec. 2, Sec. 7.2 V1-V3)
solver   residual assembly, wall-flux override (V7), CFL time step, M-stage
         Runge-Kutta (Sec. 2), wall-pressure objective

Where the paper is silent the oracle follows the readings listed in the
design notes of the repository (limiter slope form for 0/0, Harten smoothing
of all eigenvalues, diagonal-cross-product metrics, mirror slip wall,
Jameson stage coefficients 1/(M-k+1), global CFL time step).
"""

from . import gas, metrics, muscl, roe, ghosts, solver  # noqa: F401
from .solver import Problem  # noqa: F401
