"""GPU test of cfd_residual_norms_noalloc, the entry point that allocates
nothing: its partial sums live in a library-owned static device array instead
of the context workspace.  Called through the C ABI and compared with
cfd_residual_norms on two calls in a row, the second on a smaller problem
(the array keeps the first call's contents), bit for bit: both run the same
kernels over the same fixed partition."""
import ctypes

import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def _both(case):
    from paper_2012_02925_amd import capi
    from paper_2012_02925_amd.solver import Solver

    s = Solver.from_case(case, device="cuda:0")
    lib = capi.load()
    R0 = torch.empty((s.nvar, s.ncells), dtype=torch.float64, device="cuda:0")
    N0 = torch.empty(s.nvar, dtype=torch.float64, device="cuda:0")
    capi.check(lib.cfd_residual_norms(s.ctx, capi.dptr(R0), capi.dptr(N0)), s.ctx)
    R1 = torch.full_like(R0, float("nan"))
    N1 = torch.full_like(N0, float("nan"))
    capi.check(lib.cfd_residual_norms_noalloc(s.ctx, capi.dptr(R1), capi.dptr(N1)), s.ctx)
    torch.cuda.synchronize()
    out = (R0.cpu(), N0.cpu(), R1.cpu(), N1.cpu())
    s.close()
    return out


def test_noalloc_norms_match_twice_second_smaller():
    # first a larger problem (many partial sums), then a smaller one
    for case in (synth.jittered_periodic_box(dims=(64, 48, 40), seed=7),
                 synth.compression_ramp(60, 40)):
        R0, N0, R1, N1 = _both(case)
        assert torch.equal(R0, R1), case.name
        assert torch.equal(N0, N1), (case.name, N0, N1)
        assert torch.isfinite(N1).all() and (N1 >= 0).all()


def test_noalloc_rejects_null_arguments():
    from paper_2012_02925_amd import capi
    from paper_2012_02925_amd.solver import Solver

    s = Solver.from_case(synth.gaussian_bump_periodic(16, 16), device="cuda:0")
    lib = capi.load()
    N = torch.empty(4, dtype=torch.float64, device="cuda:0")
    assert lib.cfd_residual_norms_noalloc(s.ctx, None, capi.dptr(N)) == -1
    assert lib.cfd_residual_norms_noalloc(s.ctx, capi.dptr(N), None) == -1
    s.close()
