"""gpqmc_gemm_noalloc, the allocation-free GEMM entry point (descriptor in the
library's static device array), against gpqmc_debug_gemm, the entry point that
allocates its descriptor per call: the same kernels in the same tile order, so
the products agree bit for bit.  Two calls in a row on one stream, the second
with a smaller input (the array keeps the first call's descriptor until the
second overwrites it), both precisions and both tile kernels, transposed A;
requests beyond the array's tile list are refused."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2303_13403_amd import gpqmc


@pytest.mark.parametrize("prec,large,trans", [(gpqmc.FP64, False, False), (gpqmc.MIXED, False, False),
                                              (gpqmc.FP64, False, True), (gpqmc.MIXED, True, False),
                                              (gpqmc.FP64, True, False)])
def test_noalloc_gemm_equals_the_allocating_entry_point(prec, large, trans):
    dt = torch.float64 if prec == gpqmc.FP64 else torch.float32
    g = torch.Generator().manual_seed(17 + 2 * int(large) + int(trans))
    s = torch.cuda.Stream()
    outs = []
    for M, N, K in ((300, 260, 137), (70, 45, 33)):      # the second call is smaller
        A = torch.randn((K, M) if trans else (M, K), generator=g, dtype=torch.float64).to(dt).cuda()
        B = torch.randn((K, N), generator=g, dtype=torch.float64).to(dt).cuda()
        C = torch.full((M, N), float("nan"), dtype=dt, device="cuda")
        with torch.cuda.stream(s):
            gpqmc.gemm_noalloc(A, B, C, trans_a=trans, precision=prec, stream=s, large_tile=large)
        outs.append((A, B, C))
    s.synchronize()
    for A, B, C in outs:
        ref = gpqmc.debug_gemm(A, B, trans_a=trans, precision=prec, large_tile=large)
        torch.cuda.synchronize()
        assert torch.equal(C, ref)
        full = (A.T if trans else A).double() @ B.double()
        tol = 1e-13 if prec == gpqmc.FP64 else 2e-6
        assert float((C.double() - full).abs().max() / full.abs().max()) < tol


def test_noalloc_gemm_refuses_more_tiles_than_its_array_holds():
    A = torch.zeros((64 * 130, 4), dtype=torch.float64, device="cuda")
    B = torch.zeros((4, 64 * 130), dtype=torch.float64, device="cuda")
    C = torch.zeros((64 * 130, 64 * 130), dtype=torch.float64, device="cuda")
    with pytest.raises(gpqmc.GpqmcError) as e:
        gpqmc.gemm_noalloc(A, B, C, precision=gpqmc.FP64)
    assert e.value.status == gpqmc.EINVAL
