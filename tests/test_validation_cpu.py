"""Argument validation of the C ABI, on the host: every check runs before the
library touches the device, so these calls return their status without a GPU
(addresses are never dereferenced).  Limits: M up to 2^31 - 1, K and N up to
2^31 - 4 (room to pad them to a multiple of 4), lda up
to 2^21 and ldb up to 2^24 (32-bit byte offsets inside a leaf tile's slab)."""
import pytest

from paper_1205_2927_amd import fastmm

A, B, C = 0x100000, 0x40000000, 0x80000000  # disjoint fake addresses
INV, NSUP = fastmm.ERROR_INVALID_VALUE, fastmm.ERROR_NOT_SUPPORTED


@pytest.fixture(scope="module", autouse=True)
def lib():
    fastmm.load()


@pytest.mark.parametrize("args,code,msg", [
    ((-1, 4, 4, A, 4, B, 4, C, 4, 0, 1), INV, "negative"),
    ((4, 4, 8, A, 4, B, 4, C, 4, 0, 1), INV, "lda"),
    ((4, 8, 4, A, 4, B, 4, C, 8, 0, 1), INV, "ldb"),
    ((4, 8, 4, A, 4, B, 8, C, 4, 0, 1), INV, "ldc"),
    ((4, 4, 4, A, 4, B, 4, C, 4, 17, 1), INV, "depth"),
    ((4, 4, 4, 0, 4, B, 4, C, 4, 0, 1), INV, "A is NULL"),
    ((4, 4, 4, A, 4, 0, 4, C, 4, 0, 1), INV, "B is NULL"),
    ((4, 4, 4, A, 4, B, 4, 0, 4, 0, 1), INV, "C is NULL"),
    ((4, 4, 4, A, 4, B, 4, A + 8, 4, 0, 1), INV, "overlaps"),
    ((4, 4, 4, A, 4, B, 4, B + 60, 4, 0, 1), INV, "overlaps"),
    ((1 << 31, 4, 4, A, 4, B, 4, C, 4, 0, 1), NSUP, "2^31"),
    ((4, (1 << 31) - 2, 4, A, 4, B, 1 << 31, C, 1 << 31, 0, 1), NSUP, "2^31-4"),  # no room to pad N
    ((4, 4, 4, A, (1 << 21) + 1, B, 4, C, 4, 0, 1), NSUP, "lda above"),
    ((4, 4, 4, A, 4, B, (1 << 24) + 1, C, (1 << 24) + 1, 0, 1), NSUP, "ldb above"),
])
def test_gemm_rejects(args, code, msg):
    assert fastmm.gemm_raw(*args) == code
    assert msg in fastmm.last_error()


def test_gemm_ex_rejects_unknown_tile():
    assert fastmm.gemm_raw(4, 4, 4, A, 4, B, 4, C, 4, 0, 1, tile=99) == INV
    assert "tile" in fastmm.last_error()


def test_rmul_rejects():
    lib = fastmm.load()
    assert lib.fastmm_rmul(4, 4, 4, A, 4, B, 4, C, 4, -1, 1, 0) == INV
    assert lib.fastmm_rmul(4, 4, 4, A, 4, B, 4, C, 4, 1, 1, 99) == INV
    # the scaled FP16 leaf needs per-leaf scale storage the classic path lacks
    assert lib.fastmm_rmul(4, 4, 4, A, 4, B, 4, C, 4, 1, 1, fastmm.TILE_FP16X3) == NSUP
    assert lib.fastmm_rmul(4, 4, 4, A, 2, B, 4, C, 4, 1, 1, 0) == INV


def test_batched_rejects_atomically():
    # the second problem is invalid: the whole call fails before any work
    rc = fastmm.gemm_batched_raw([4, 4], [4, 4], [4, 4], [A, A + 4096], [4, 4], [B, B + 4096],
                                 [4, 2], [C, C + 4096], [4, 4])
    assert rc == INV
    assert "problem 1" in fastmm.last_error() or "ldb" in fastmm.last_error()
