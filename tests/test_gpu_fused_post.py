"""The last level's post-additions fused into the FP32 leaf's epilogue
(FASTMM_FUSED_POST=1): the seven products of each last-level node run as
seven launches, each adding its product into the node's result quadrants in
the order of the post-addition chains, so the result must equal the unfused
schedule's bit for bit, on the level-wise path and on the pipelined host
path, and match the oracle."""
import numpy as np
import pytest

from oracle import checks, classic
from oracle import winograd as W
from tests.gpu_util import dev, empty_dev, host, ints, say, uniform

pytestmark = pytest.mark.gpu


def _pair(fastmm, monkeypatch, m, k, n, depth, A, B):
    monkeypatch.delenv("FASTMM_FUSED_POST", raising=False)
    C0 = empty_dev(m, n)
    fastmm.gemm(m, n, k, dev(A), dev(B), C0, depth=depth, leaf=1)
    s0 = fastmm.get_stats()
    monkeypatch.setenv("FASTMM_FUSED_POST", "1")
    C1 = empty_dev(m, n)
    fastmm.gemm(m, n, k, dev(A), dev(B), C1, depth=depth, leaf=1)
    s1 = fastmm.get_stats()
    monkeypatch.delenv("FASTMM_FUSED_POST")
    return host(C0), host(C1), s0, s1


@pytest.mark.parametrize("m,k,n,depth", [(512, 512, 512, 1), (1000, 700, 900, 1), (768, 640, 896, 2),
                                         (1030, 1031, 1029, 3), (333, 201, 257, 3), (1024, 1024, 1024, 4)])
def test_fused_post_equals_unfused(fastmm, monkeypatch, m, k, n, depth):
    say(f"fused post-additions {m}x{k}x{n} depth={depth}")
    A = uniform(8301 + m, m, k)
    B = uniform(8302 + n, k, n)
    c0, c1, s0, s1 = _pair(fastmm, monkeypatch, m, k, n, depth, A, B)
    assert s0["depth"] == s1["depth"] == depth
    assert s1["launches"] > s0["launches"]  # seven leaf launches
    assert np.array_equal(c0, c1)
    assert checks.rel_frob(c1, classic.gemm(A, B)) <= 1e-4


@pytest.mark.parametrize("m,k,n,depth", [(257, 131, 383, 2), (97, 301, 45, 3), (640, 512, 768, 3)])
def test_fused_post_certified_exact(fastmm, monkeypatch, m, k, n, depth):
    A = ints(8311 + m, m, k)
    B = ints(8312 + n, k, n)
    cert = W.Certificate()
    ref = W.winograd(A.astype(np.int64), B.astype(np.int64), depth, 1, cert)
    assert cert.exact_in_fp32
    c0, c1, s0, s1 = _pair(fastmm, monkeypatch, m, k, n, depth, A, B)
    assert np.array_equal(c1.astype(np.int64), ref)
    assert np.array_equal(c0, c1)


def test_fused_post_pipelined_host(fastmm, monkeypatch):
    # Host operands: every piece of the pipelined top level is a depth-2
    # product whose last level is fused.
    import torch
    n = 2048
    A = uniform(8321, n, n)
    B = uniform(8322, n, n)
    Ah = torch.from_numpy(A).pin_memory()
    Bh = torch.from_numpy(B).pin_memory()
    outs = []
    for fused in ("0", "1"):
        monkeypatch.setenv("FASTMM_FUSED_POST", fused)
        Ch = torch.full((n, n), float("nan")).pin_memory()
        fastmm.gemm(n, n, n, Ah, Bh, Ch, depth=3, leaf=1)
        assert fastmm.get_stats()["depth"] == 3
        outs.append(Ch.numpy().copy())
    assert np.array_equal(outs[0], outs[1])
    assert checks.rel_frob(outs[1], classic.gemm(A, B)) <= 1e-4
