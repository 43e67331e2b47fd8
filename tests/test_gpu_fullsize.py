"""Parity at the benchmark's full sizes: square n = 19456 with the operands in
HBM (the launch configuration bench.py times for its headline: one
level-wise call, one grouped leaf launch) and with the operands in pinned
host memory (transfers inside the call, the benchmark's pinned_host block),
and the rectangular 19456 x 16384 x 12288 product.  The oracle cannot afford
the full product on every run, so it checks seeded sampled rows exactly
(FP64-accumulated) and Freivalds' probe C x = A (B x)."""
import numpy as np
import pytest

import synthgen
from oracle import checks
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

TOL = 1e-4


def _pinned(shape):
    import torch
    return torch.empty(shape, dtype=torch.float32, pin_memory=True)


def _check(fastmm, M, N, K, depth, leaf, seed_a, seed_b, rows=24, device=False, tile=0, tol=TOL):
    A = _pinned((M, K))
    B = _pinned((K, N))
    C = _pinned((M, N))
    synthgen.fill_uniform_pm1(seed_a, M, K, A.data_ptr())
    synthgen.fill_uniform_pm1(seed_b, K, N, B.data_ptr())
    C.fill_(float("nan"))
    say(f"full size {M}x{K}x{N} depth={depth} leaf={leaf} device={device} tile={tile}")
    if device:
        dA, dB, dC = A.to("cuda"), B.to("cuda"), C.to("cuda")
        fastmm.gemm(M, N, K, dA, dB, dC, depth=depth, leaf=leaf, tile=tile)
        st = fastmm.get_stats()
        C.copy_(dC)
        del dA, dB, dC
    else:
        fastmm.gemm(M, N, K, A, B, C, depth=depth, leaf=leaf, tile=tile)
        st = fastmm.get_stats()
    An, Bn, Cn = A.numpy(), B.numpy(), C.numpy()
    assert np.isfinite(Cn).all()
    r = synthgen.row_sample(seed_a + 7, M, rows)
    e_rows = checks.sampled_rows_rel(Cn, An, Bn, r)
    e_fv = checks.freivalds_rel(Cn, An, Bn, synthgen.signs_pm1(seed_b + 7, N))
    say(f"  depth={st['depth']} sampled-rows rel={e_rows:.3e} freivalds rel={e_fv:.3e}")
    assert e_rows <= tol and e_fv <= tol
    return st


def test_headline_square_19456_depth3_device(fastmm):
    st = _check(fastmm, 19456, 19456, 19456, 3, 1024, 1001 + 3, 2001 + 3, device=True)
    assert st["depth"] == 3
    # level-wise: all 343 leaves in one grouped launch
    assert st["leaves"] == 343 and st["leaf_launches"] == 1
    assert abs(st["leaf_flops"] - 2 * 19456**3 * (7 / 8) ** 3) < 1e-6 * 2 * 19456**3


def test_plain_square_19456_device(fastmm):
    st = _check(fastmm, 19456, 19456, 19456, 0, 1024, 1001 + 3, 2001 + 3, rows=12, device=True)
    assert st["depth"] == 0 and st["leaf_launches"] == 1


def test_headline_square_19456_depth3_pinned(fastmm):
    st = _check(fastmm, 19456, 19456, 19456, 3, 1024, 1001 + 3, 2001 + 3)
    assert st["depth"] == 3
    # 7 top-level products in four row bands x two column bands, each piece
    # a depth-2 product of 49 leaves, one grouped leaf launch per piece
    assert st["leaves"] == 8 * 7 * 49 and st["leaf_launches"] == 56
    assert abs(st["leaf_flops"] - 2 * 19456**3 * (7 / 8) ** 3) < 1e-6 * 2 * 19456**3


@pytest.mark.parametrize("depth", [0, 2, 4])
def test_square_19456_other_depths_pinned(fastmm, depth):
    st = _check(fastmm, 19456, 19456, 19456, depth, 1024 if depth < 4 else 1, 1001 + 3, 2001 + 3,
                rows=12)
    assert st["depth"] == depth


@pytest.mark.parametrize("depth,leaf", [(2, 1024), (3, 1024), (4, 768)])
def test_rectangular_19456x16384x12288_pinned(fastmm, depth, leaf):
    st = _check(fastmm, 19456, 12288, 16384, depth, leaf, 1001 + 3, 2001 + 3, rows=12)
    assert st["depth"] == depth


@pytest.mark.parametrize("tile,depth,tol", [(8, 0, 2e-5), (8, 2, 1e-4), (9, 0, 5e-6), (9, 2, 2e-5)])
def test_precision_forms_square_19456_device(fastmm, tile, depth, tol):
    # The precision forms at the benchmark's size (its precision_forms
    # block): split BF16 (tile 8) and scaled split FP16 (tile 9) at depth 0
    # and at depth 2 with the fused last-level passes.
    st = _check(fastmm, 19456, 19456, 19456, depth, 1024, 1001 + 3, 2001 + 3, rows=8, device=True,
                tile=tile, tol=tol)
    assert st["depth"] == depth and st["tile"] == tile

