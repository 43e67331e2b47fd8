"""Parity of the individual GPU kernels against the oracle, through the C ABI.

Pre- and post-additions: each output element is one fixed FP32 chain, so
the GPU must equal the oracle's FP32 evaluation of the same chain bit for
bit.  Leaf product (depth 0): tolerance against the FP64 classic product on
uniform inputs, bit-exact on inputs whose every partial sum is an exactly
representable integer, and bit-exact for A*I = A."""
import numpy as np
import pytest

from oracle import checks, classic
from oracle import winograd as W
from tests.gpu_util import dev, empty_dev, host, ints, say, uniform

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("rows,cols", [(64, 64), (96, 128), (33, 17), (7, 9), (1, 1), (256, 516), (130, 258)])
@pytest.mark.parametrize("side", [0, 1])
def test_preadd_bit_exact(fastmm, rows, cols, side):
    say(f"preadd side={side} {rows}x{cols}")
    X = uniform(11 + rows + side, rows, cols)
    h_r, h_c = W.half_up(rows), W.half_up(cols)
    out = empty_dev(4 * h_r, h_c)
    fastmm.preadd(side, rows, cols, dev(X), out)
    got = host(out).reshape(4, h_r, h_c)
    q = W.quadrants(X)
    ref = W.preadd_a(*q) if side == 0 else W.preadd_b(*q)
    for i in range(4):
        assert ref[i].dtype == np.float32
        assert np.array_equal(got[i], ref[i]), f"output {i + 1}"


def test_preadd_strided_view(fastmm):
    # Parent operand with a leading dimension larger than its width.
    big = uniform(21, 40, 100)
    X = big[:, :60]
    out = empty_dev(4 * 20, 30)
    import torch
    t = dev(big)
    fastmm.preadd(0, 40, 60, t.data_ptr(), out, ldx=100)
    got = host(out).reshape(4, 20, 30)
    ref = W.preadd_a(*W.quadrants(X))
    for i in range(4):
        assert np.array_equal(got[i], ref[i])


@pytest.mark.parametrize("h_r,h_c,rows,cols", [(32, 32, 64, 64), (17, 9, 33, 17), (17, 9, 34, 18),
                                               (64, 128, 128, 256), (1, 1, 1, 1), (5, 12, 9, 23),
                                               # odd h_c with many rows: the last partial group of
                                               # a left quadrant and the first group of the right
                                               # one fall in different wavefronts
                                               (100, 65, 200, 130), (50, 33, 99, 65), (301, 7, 602, 13)])
def test_postadd_bit_exact(fastmm, h_r, h_c, rows, cols):
    say(f"postadd {h_r}x{h_c} -> {rows}x{cols}")
    P = uniform(31 + h_r, 7 * h_r, h_c)
    C = empty_dev(rows, cols, fill=-7.0)
    fastmm.postadd(h_r, h_c, dev(P), C, rows, cols)
    C11, C12, C21, C22 = W.postadd(*P.reshape(7, h_r, h_c))
    ref = W.assemble(C11, C12, C21, C22, rows, cols)
    assert ref.dtype == np.float32
    assert np.array_equal(host(C), ref)


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 5, 6, 7, 9])
def test_leaf_n512_uniform(fastmm, tile):
    say(f"leaf n=512 tile={tile}")
    n = 512
    A = uniform(1001 + 1, n, n)
    B = uniform(2001 + 1, n, n)
    C = empty_dev(n, n)
    fastmm.gemm(n, n, n, dev(A), dev(B), C, depth=0, tile=tile)
    err = checks.rel_frob(host(C), classic.gemm(A, B))
    say(f"  rel_frob={err:.3e}")
    assert err <= 2e-6


# tiles 8 and 9 (split BF16 / scaled split FP16) are exact on these small
# integers too: hi holds them exactly and lo is zero.
@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9])
@pytest.mark.parametrize("m,k,n", [(257, 131, 383), (1, 1, 1), (33, 65, 17), (130, 7, 260),
                                   (300, 1000, 5), (64, 64, 64), (129, 257, 127)])
def test_leaf_ragged_certified_exact(fastmm, tile, m, k, n):
    say(f"leaf ragged {m}x{k}x{n} tile={tile}")
    A = ints(41 + m, m, k, -2, 2)
    B = ints(42 + n, k, n, -2, 2)
    assert k * 4 < 2**24  # every partial sum is an exact FP32 integer
    C = empty_dev(m, n)
    fastmm.gemm(m, n, k, dev(A), dev(B), C, depth=0, tile=tile)
    ref = classic.gemm(A.astype(np.int64), B.astype(np.int64))
    assert np.array_equal(host(C).astype(np.int64), ref)


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9])
@pytest.mark.parametrize("m,k,n", [(300, 1000, 260), (129, 36, 132), (1000, 4, 4),
                                   (5, 20, 1028), (257, 132, 388)])
def test_leaf_vector_path_ragged_exact(fastmm, tile, m, k, n):
    # K and N multiples of 4 with aligned rows: the 16-byte load path (slabs
    # loaded straight into LDS for 16-deep tiles), with partial tiles in M
    # and N and a partial last K-slab, all zero-filled by the buffer loads.
    say(f"leaf vector-path ragged {m}x{k}x{n} tile={tile}")
    A = ints(43 + m, m, k, -2, 2)
    B = ints(44 + n, k, n, -2, 2)
    C = empty_dev(m, n)
    fastmm.gemm(m, n, k, dev(A), dev(B), C, depth=0, tile=tile)
    ref = classic.gemm(A.astype(np.int64), B.astype(np.int64))
    assert np.array_equal(host(C).astype(np.int64), ref)


def test_leaf_identity_bit_exact(fastmm):
    n = 384
    A = uniform(51, n, n)
    I = np.eye(n, dtype=np.float32)
    C = empty_dev(n, n)
    fastmm.gemm(n, n, n, dev(A), dev(I), C, depth=0)
    assert np.array_equal(host(C), A)
    fastmm.gemm(n, n, n, dev(I), dev(A), C, depth=0)
    assert np.array_equal(host(C), A)


def test_leaf_unaligned_leading_dims(fastmm):
    # lda, ldb, ldc odd: the scalar load path.
    import torch
    m, k, n = 70, 45, 53
    Abig = uniform(61, m, k + 3)
    Bbig = uniform(62, k, n + 1)
    A = dev(Abig)
    B = dev(Bbig)
    C = torch.full((m, n + 5), float("nan"), device="cuda")
    fastmm.gemm(m, n, k, A.data_ptr(), B.data_ptr(), C.data_ptr(), depth=0,
                lda=k + 3, ldb=n + 1, ldc=n + 5)
    got = host(C)
    ref = classic.gemm(Abig[:, :k], Bbig[:, :n])
    assert checks.rel_frob(got[:, :n], ref) < 2e-6
    assert np.all(np.isnan(got[:, n:]))  # nothing written outside C
