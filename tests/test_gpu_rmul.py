"""Parity of fastmm_rmul, the classic eight-product recursion of Table 1,
against the oracle's own Table 1 recursion and the classic product.

Integer inputs in {-1, 0, 1} keep every FP32 partial sum an exact integer,
so those cases are compared bit for bit.  Uniform inputs: relative Frobenius
error against the FP64 classic product at most 5e-6 (FP32 accumulation over
K <= 1536 plus 2^depth FP32 chunk additions)."""
import numpy as np
import pytest

from oracle import checks, classic
from oracle import winograd as W
from tests.gpu_util import dev, empty_dev, host, ints, say, uniform

pytestmark = pytest.mark.gpu

TOL_RMUL = 5e-6


@pytest.mark.parametrize("m,k,n,depth", [(257, 131, 383, 2), (33, 65, 17, 3), (101, 99, 103, 4),
                                         (200, 64, 130, 1), (3, 3, 3, 1), (640, 640, 640, 0)])
@pytest.mark.parametrize("tile", [0, 3])
def test_rmul_ragged_exact(fastmm, m, k, n, depth, tile):
    say(f"rmul ragged {m}x{k}x{n} depth={depth} tile={tile}")
    A = ints(171 + m, m, k)
    B = ints(172 + n, k, n)
    ref = W.rmul(A.astype(np.int64), B.astype(np.int64), depth, 1)
    assert np.array_equal(ref, classic.gemm(A.astype(np.int64), B.astype(np.int64)))
    C = empty_dev(m, n)
    fastmm.rmul(m, n, k, dev(A), dev(B), C, depth=depth, leaf=1, tile=tile)
    st = fastmm.get_stats()
    d = W.effective_depth(m, k, n, depth, 1)
    assert st["depth"] == d
    assert st["leaf_launches"] == 2 ** d
    assert st["leaves"] == 8 ** d
    assert st["leaf_flops"] == 2.0 * m * n * k
    assert np.array_equal(host(C).astype(np.int64), ref)


@pytest.mark.parametrize("n,depth,leaf,tile", [(1024, 2, 128, 0), (1536, 3, 128, 0),
                                               (1000, 2, 64, 2), (768, 1, 256, 6)])
def test_rmul_uniform(fastmm, n, depth, leaf, tile):
    say(f"rmul uniform n={n} depth={depth} leaf={leaf} tile={tile}")
    A = uniform(3101, n, n)
    B = uniform(3102, n, n)
    C = empty_dev(n, n)
    fastmm.rmul(n, n, n, dev(A), dev(B), C, depth=depth, leaf=leaf, tile=tile)
    assert fastmm.get_stats()["depth"] == W.effective_depth(n, n, n, depth, leaf)
    err = checks.rel_frob(host(C), classic.gemm(A, B))
    say(f"  rel_frob={err:.3e}")
    assert err <= TOL_RMUL


def test_rmul_depth0_equals_classic_leaf_bitwise(fastmm):
    # one chunk, no accumulation: the same leaf kernel as fastmm_gemm at depth 0
    m, k, n = 515, 387, 641
    A, B = uniform(3201, m, k), uniform(3202, k, n)
    C1, C2 = empty_dev(m, n), empty_dev(m, n)
    fastmm.rmul(m, n, k, dev(A), dev(B), C1, depth=0, tile=0)
    fastmm.gemm(m, n, k, dev(A), dev(B), C2, depth=0, tile=0)
    assert np.array_equal(host(C1), host(C2))


def test_rmul_host_operands_and_strides(fastmm):
    import torch
    m, k, n = 700, 520, 610
    A = ints(3301, m, k + 9)
    B = ints(3302, k, n + 5)
    Ah = torch.from_numpy(A).pin_memory()[:, :k]
    Bh = torch.from_numpy(B)[:, :n]          # pageable, strided
    Ch = torch.full((m, n + 3), float("nan")).pin_memory()[:, :n]
    fastmm.rmul(m, n, k, Ah, Bh, Ch, depth=2, leaf=64)
    ref = classic.gemm(A[:, :k].astype(np.int64), B[:, :n].astype(np.int64))
    assert np.array_equal(Ch.numpy().astype(np.int64), ref)


def test_rmul_empty_and_k0(fastmm):
    import torch
    C = empty_dev(5, 7)
    A = torch.zeros((5, 1), device="cuda")
    B = torch.zeros((1, 7), device="cuda")
    fastmm.rmul(5, 7, 0, A, B, C, depth=2, leaf=1, lda=1, ldb=7)
    assert np.all(host(C) == 0)
    fastmm.rmul(0, 7, 3, A, B, C, depth=2, leaf=1, lda=3, ldb=7)  # no-op


def test_rmul_invalid_args(fastmm):
    A = empty_dev(8, 8, 0)
    with pytest.raises(fastmm.FastmmError):
        fastmm.rmul(8, 8, 8, A, A, A, depth=-1)
    with pytest.raises(fastmm.FastmmError):
        fastmm.rmul(8, 8, 8, A, A, A, depth=1, tile=99)
    with pytest.raises(fastmm.FastmmError):
        fastmm.rmul(8, 8, 8, A, A, A, depth=1, ldb=4)


def test_rmul_bf16x3_tile(fastmm):
    n = 1024
    A, B = uniform(3401, n, n), uniform(3402, n, n)
    C = empty_dev(n, n)
    fastmm.rmul(n, n, n, dev(A), dev(B), C, depth=2, leaf=128, tile=8)
    err = checks.rel_frob(host(C), classic.gemm(A, B))
    say(f"rmul bf16x3 rel_frob={err:.3e}")
    assert err <= 2e-5
