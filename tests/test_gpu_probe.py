"""GPU test of the streaming-bandwidth probe the bench uses as its practical
HBM ceiling: the kernel really reads every element of every input array and
writes every output array (dst_b[e] = sum_a src_a[e] + b), for both access
widths and a length that is not a multiple of the workgroup size."""
import ctypes

import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("reads,writes", [(4, 1), (3, 1), (20, 5), (15, 5), (1, 1)])
@pytest.mark.parametrize("vec", [1, 2])
def test_stream_probe_moves_every_element(reads, writes, vec):
    from paper_2012_02925_amd import capi
    lib = capi.load()
    n = 1000006  # even, not a multiple of 256
    g = torch.Generator().manual_seed(reads * 10 + vec)
    src = torch.rand(reads * n, dtype=torch.float64, generator=g).to("cuda:0")
    dst = torch.full((writes * n,), float("nan"), dtype=torch.float64, device="cuda:0")
    ms = ctypes.c_double()
    st = torch.cuda.current_stream()
    capi.check(lib.cfd_stream_probe(reads, writes, vec, capi.dptr(src), capi.dptr(dst), n, 2,
                                    ctypes.c_void_p(st.cuda_stream), ctypes.byref(ms)))
    total = src.reshape(reads, n).sum(0)
    out = dst.reshape(writes, n)
    for b in range(writes):
        torch.testing.assert_close(out[b], total + b, rtol=1e-14, atol=1e-13)
    assert ms.value > 0.0


def test_stream_probe_rejects_bad_arguments():
    from paper_2012_02925_amd import capi
    lib = capi.load()
    src = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    dst = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    ms = ctypes.c_double()
    assert lib.cfd_stream_probe(2, 1, 1, capi.dptr(src), capi.dptr(dst), 4, 1, None, ctypes.byref(ms)) == -1
    assert lib.cfd_stream_probe(1, 1, 2, capi.dptr(src), capi.dptr(dst), 3, 1, None, ctypes.byref(ms)) == -1
    assert lib.cfd_stream_probe(1, 1, 1, None, capi.dptr(dst), 4, 1, None, ctypes.byref(ms)) == -1
