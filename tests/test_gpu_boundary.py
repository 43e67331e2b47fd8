"""The MM-queue calls of the boundary (Section 3.3: one command queue and one
set of buffers per device, set up once and reused): products run on a
caller's stream after the work queued on it, and the library can be torn
down and built again."""
import numpy as np
import pytest

from oracle import checks, classic
from tests.gpu_util import dev, empty_dev, host, say, uniform

pytestmark = pytest.mark.gpu


def test_set_stream_runs_after_queued_work(fastmm):
    import torch
    n = 1536
    A = uniform(8201, n, n)
    B = uniform(8202, n, n)
    dA, dB = dev(A), dev(B)
    ref = empty_dev(n, n)
    fastmm.gemm(n, n, n, dA, dB, ref, depth=2, leaf=128)  # on the library's own stream
    A2 = torch.zeros_like(dA)
    B2 = torch.zeros_like(dB)
    C = empty_dev(n, n)
    big = torch.ones(1 << 26, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    try:
        with torch.cuda.stream(s):
            # keep the side stream busy, then produce the operands on it
            for _ in range(40):
                big.mul_(1.0)
            A2.copy_(dA)
            B2.copy_(dB)
        say("gemm on a caller's side stream after queued work")
        fastmm.set_stream(s)
        fastmm.gemm(n, n, n, A2, B2, C, depth=2, leaf=128)
        # the call returned: its work on the side stream is done
        assert s.query()
        got = host(C)
        assert np.array_equal(got, host(ref))
        assert checks.rel_frob(got, classic.gemm(A, B)) <= 1e-4
    finally:
        fastmm.set_stream(None)
    C2 = empty_dev(n, n)
    fastmm.gemm(n, n, n, dA, dB, C2, depth=2, leaf=128)
    assert np.array_equal(host(C2), host(ref))


def test_finalize_then_fresh_calls(fastmm):
    import torch
    n = 1024
    A = uniform(8211, n, n)
    B = uniform(8212, n, n)
    dA, dB = dev(A), dev(B)
    C1 = empty_dev(n, n)
    fastmm.gemm(n, n, n, dA, dB, C1, depth=3, leaf=64)
    shapes = [(256, 320, 192), (384, 512, 448)]
    As = [dev(uniform(8220 + i, m, k)) for i, (m, k, nn) in enumerate(shapes)]
    Bs = [dev(uniform(8230 + i, k, nn)) for i, (m, k, nn) in enumerate(shapes)]
    Cb1 = [empty_dev(m, nn) for (m, k, nn) in shapes]
    fastmm.gemm_batched(As, Bs, Cb1, depth=[2, 2], leaf=[1, 1])
    s = torch.cuda.Stream()
    fastmm.set_stream(s)
    say("finalize (twice), then fresh calls")
    fastmm.finalize()
    fastmm.finalize()
    # everything is built again: same results, bit for bit, on the library's
    # own stream (finalize forgets the caller's stream)
    C2 = empty_dev(n, n)
    fastmm.gemm(n, n, n, dA, dB, C2, depth=3, leaf=64)
    st = fastmm.get_stats()
    assert st["depth"] == 3 and st["workspace_bytes"] > 0
    assert np.array_equal(host(C2), host(C1))
    assert checks.rel_frob(host(C2), classic.gemm(A, B)) <= 1e-4
    Cb2 = [empty_dev(m, nn) for (m, k, nn) in shapes]
    fastmm.gemm_batched(As, Bs, Cb2, depth=[2, 2], leaf=[1, 1])
    assert fastmm.get_stats()["graph_replayed"] == 0  # the graph cache was released
    for a, b in zip(Cb1, Cb2):
        assert np.array_equal(host(a), host(b))
    # host operands (staging buffers rebuilt too)
    Ah = torch.from_numpy(A).pin_memory()
    Bh = torch.from_numpy(B).pin_memory()
    Ch = torch.full((n, n), float("nan")).pin_memory()
    fastmm.gemm(n, n, n, Ah, Bh, Ch, depth=3, leaf=64)
    assert checks.rel_frob(Ch.numpy(), classic.gemm(A, B)) <= 1e-4


def test_set_stream_host_operands_two_compute_streams(fastmm):
    # Host operands on a caller's side stream: the staged path's other
    # streams (copies in and out, the second compute stream) start after the
    # work queued on it and it waits for them, so the call returns with the
    # side stream drained and the result equals the default stream's.
    import torch
    M, K, N = 3000, 2000, 8195
    A = uniform(8241, M, K)
    B = uniform(8242, K, N)
    Ah = torch.from_numpy(A).pin_memory()
    Bh = torch.from_numpy(B).pin_memory()
    ref = torch.full((M, N), float("nan")).pin_memory()
    fastmm.gemm(M, N, K, Ah, Bh, ref, depth=2, leaf=1)
    big = torch.ones(1 << 26, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    Ch = torch.full((M, N), float("nan")).pin_memory()
    try:
        with torch.cuda.stream(s):
            for _ in range(40):
                big.mul_(1.0)
        say("pinned gemm on a caller's side stream after queued work")
        fastmm.set_stream(s)
        fastmm.gemm(M, N, K, Ah, Bh, Ch, depth=2, leaf=1)
        assert s.query()
    finally:
        fastmm.set_stream(None)
    assert np.array_equal(Ch.numpy(), ref.numpy())
    assert checks.rel_frob(Ch.numpy()[:64], classic.gemm(A[:64], B)) <= 1e-4
