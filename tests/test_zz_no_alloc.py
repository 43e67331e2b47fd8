"""fastmm_gemm_noalloc (the entry point for callers that cannot allocate)
through the C ABI: the same product as fastmm_gemm, bit for bit, and within
the oracle's tolerance, on two calls in a row (the second smaller), with no
change in free device memory; products that need more than the static
workspace are rejected before anything is written."""
import numpy as np
import pytest

from oracle import checks, classic
from tests.gpu_util import dev, empty_dev, host, say, uniform

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _pair(fastmm, m, k, n, depth, leaf, seed):
    import torch
    A = uniform(seed, m, k)
    B = uniform(seed + 1, k, n)
    dA, dB = dev(A), dev(B)
    ref = empty_dev(m, n)
    fastmm.gemm(m, n, k, dA, dB, ref, depth=depth, leaf=leaf)
    ref_stats = fastmm.get_stats()
    C = empty_dev(m, n)
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    say(f"noalloc {m}x{k}x{n} depth={depth} leaf={leaf}")
    fastmm.gemm_noalloc(m, n, k, dA, dB, C, depth=depth, leaf=leaf)
    free1, _ = torch.cuda.mem_get_info()
    st = fastmm.get_stats()
    return A, B, host(C), host(ref), st, ref_stats, free0, free1


def test_noalloc_matches_gemm_two_calls(fastmm):
    for (m, k, n, depth, leaf, seed) in [(1536, 1024, 1280, 2, 128, 8101), (520, 300, 388, 1, 64, 8111)]:
        A, B, got, ref, st, rst, free0, free1 = _pair(fastmm, m, k, n, depth, leaf, seed)
        assert st["depth"] == rst["depth"] == depth
        assert st["leaves"] == 7 ** depth
        assert np.array_equal(got, ref)
        assert checks.rel_frob(got, classic.gemm(A, B)) <= TOL
        assert free1 == free0  # the call took no device memory
        assert 0 < st["workspace_bytes"] <= fastmm.NOALLOC_WORKSPACE_BYTES


def test_noalloc_depth0_and_planner_rule(fastmm):
    import torch
    n = 512
    A = uniform(8121, n, n)
    B = uniform(8122, n, n)
    C = empty_dev(n, n)
    fastmm.gemm_noalloc(n, n, n, dev(A), dev(B), C, depth=0)
    assert checks.rel_frob(host(C), classic.gemm(A, B)) <= 2e-6
    C2 = empty_dev(n, n)
    fastmm.gemm_noalloc(n, n, n, dev(A), dev(B), C2, depth=-1)  # fixed rule: depth 0, 64x64 tiles
    assert fastmm.get_stats()["depth"] == 0
    assert checks.rel_frob(host(C2), classic.gemm(A, B)) <= 2e-6
    # K == 0: C is set to zero
    C3 = torch.full((64, 32), 3.0, device="cuda")
    fastmm.gemm_noalloc(64, 32, 0, dev(np.zeros((64, 4), np.float32)), dev(np.zeros((4, 32), np.float32)),
                        C3, depth=0, lda=4)
    assert torch.all(C3 == 0).item()


def test_noalloc_rejects_what_needs_allocation(fastmm):
    import torch
    n = 8192
    A = torch.zeros((n, n), device="cuda")
    B = torch.zeros((n, n), device="cuda")
    C = torch.full((n, n), 5.0, device="cuda")
    # depth 3 at n = 8192 needs far more than the static workspace
    rc = fastmm.gemm_noalloc_raw(n, n, n, A.data_ptr(), n, B.data_ptr(), n, C.data_ptr(), n, 3, 512)
    assert rc == fastmm.ERROR_OUT_OF_MEMORY
    assert "static workspace" in fastmm.last_error()
    assert torch.all(C == 5.0).item()
    # host operands and misaligned device operands need staging copies
    h = torch.zeros((64, 64)).pin_memory()
    rc = fastmm.gemm_noalloc_raw(64, 64, 64, h.data_ptr(), 64, h.data_ptr(), 64,
                                 torch.zeros((64, 64)).pin_memory().data_ptr(), 64, 0, 1)
    assert rc == fastmm.ERROR_NOT_SUPPORTED
    Cm = torch.full((63, 63), 5.0, device="cuda")
    rc = fastmm.gemm_noalloc_raw(63, 63, 63, A.data_ptr(), 63, B.data_ptr(), 63, Cm.data_ptr(), 63, 0, 1)
    assert rc == fastmm.ERROR_NOT_SUPPORTED
    assert torch.all(Cm == 5.0).item()
