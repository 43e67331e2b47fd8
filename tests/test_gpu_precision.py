"""Precision form of the leaf (split BF16, "bf16x3"): products of hi/lo BF16
halves accumulated in FP32 on the BF16 matrix cores; quadrant additions stay
FP32.  Checked against the FP64 oracle: exact on integers the split
represents exactly, and the relative error reported per result for uniform
and log-uniform inputs (the accuracy is about 2^-16 per product instead of
FP32's 2^-24, so the bounds here are looser than the FP32 leaf's)."""
import numpy as np
import pytest

import synthgen
from oracle import checks, classic
from oracle import winograd as W
from tests.gpu_util import dev, empty_dev, host, ints, say, uniform

pytestmark = pytest.mark.gpu
BF = 8  # FASTMM_TILE_BF16X3_128x128


@pytest.mark.parametrize("m,k,n,depth", [(256, 256, 256, 0), (257, 131, 383, 0), (300, 200, 100, 2),
                                         (512, 512, 512, 3)])
def test_bf16x3_exact_on_small_integers(fastmm, m, k, n, depth):
    # Integers of magnitude <= 3 have an exact BF16 hi part and zero lo part;
    # with every partial sum below 2^24 the result is exact.
    A = ints(141 + m, m, k, -3, 3)
    B = ints(142 + n, k, n, -3, 3)
    cert = W.Certificate()
    leaf_max = [0]

    def leaf(a, b):  # record the largest leaf operand: it must be exact in BF16
        leaf_max[0] = max(leaf_max[0], int(np.abs(a).max(initial=0)), int(np.abs(b).max(initial=0)))
        return classic.gemm(a, b)

    ref = W.winograd(A.astype(np.int64), B.astype(np.int64), depth, 1, cert, leaf_fn=leaf)
    assert cert.exact_in_fp32 and leaf_max[0] <= 256
    C = empty_dev(m, n)
    fastmm.gemm(m, n, k, dev(A), dev(B), C, depth=depth, leaf=1, tile=BF)
    assert np.array_equal(host(C).astype(np.int64), ref)


@pytest.mark.parametrize("dist", ["uniform", "loguniform"])
@pytest.mark.parametrize("n,depth,bound", [(512, 0, 5e-5), (1024, 2, 2e-4), (768, 1, 1e-4)])
def test_bf16x3_error_vs_oracle(fastmm, dist, n, depth, bound):
    gen = synthgen.uniform_pm1 if dist == "uniform" else synthgen.loguniform
    A = gen(1001 + 4, n, n)
    B = gen(2001 + 4, n, n)
    C = empty_dev(n, n)
    fastmm.gemm(n, n, n, dev(A), dev(B), C, depth=depth, leaf=1, tile=BF)
    ref = classic.gemm(A, B)
    e = checks.rel_frob(host(C), ref)
    # the FP32 leaf on the same inputs, for the record
    C32 = empty_dev(n, n)
    fastmm.gemm(n, n, n, dev(A), dev(B), C32, depth=depth, leaf=1, tile=0)
    e32 = checks.rel_frob(host(C32), ref)
    say(f"  bf16x3 {dist} n={n} depth={depth}: rel_frob={e:.3e} (fp32 leaf {e32:.3e})")
    assert e <= bound


@pytest.mark.parametrize("n", [8192, 16384])
def test_config4_depth2_sampled(fastmm, n):
    # n = 8192 and 16384, depth 2, both input distributions.
    for dist, gen in [("uniform", synthgen.uniform_pm1), ("loguniform", synthgen.loguniform)]:
        A = gen(1001 + 4, n, n)
        B = gen(2001 + 4, n, n)
        C = empty_dev(n, n)
        fastmm.gemm(n, n, n, dev(A), dev(B), C, depth=2, leaf=1, tile=BF)
        got = host(C)
        rows = synthgen.row_sample(7008, n, 12)
        e_rows = checks.sampled_rows_rel(got, A, B, rows)
        e_fv = checks.freivalds_rel(got, A, B, synthgen.signs_pm1(7009, n))
        say(f"  split-BF16 {dist} n={n}: sampled-rows rel={e_rows:.3e} freivalds rel={e_fv:.3e}")
        assert e_rows <= 2e-4 and e_fv <= 2e-4
