"""Precision forms of the leaf: split BF16 ("bf16x3", hi/lo BF16 halves on
the BF16 matrix cores) and scaled split FP16 ("fp16x3", each row of a leaf's
A and column of its B scaled by a power of two, then split into hi/lo FP16
halves on the FP16 matrix cores); products accumulate in FP32 and the
quadrant additions stay FP32.  Checked against the FP64 oracle: exact on
integers the split represents exactly, the relative error reported per
result for uniform and log-uniform inputs (bf16x3: about 2^-16 per product;
fp16x3: about 2^-21, the FP32 leaf's level), and for fp16x3 the scaling
itself: exact equivariance under power-of-two row and column scalings, and
inputs far outside FP16's range."""
import numpy as np
import pytest

import synthgen
from oracle import checks, classic, split
from oracle import winograd as W
from tests.gpu_util import dev, empty_dev, host, ints, say, uniform

pytestmark = pytest.mark.gpu
BF = 8  # FASTMM_TILE_BF16X3
FP = 9  # FASTMM_TILE_FP16X3


@pytest.mark.parametrize("tile", [BF, FP])
@pytest.mark.parametrize("m,k,n,depth", [(256, 256, 256, 0), (257, 131, 383, 0), (300, 200, 100, 2),
                                         (512, 512, 512, 3)])
def test_split_exact_on_small_integers(fastmm, m, k, n, depth, tile):
    # Integers of magnitude <= 256 have an exact BF16 (and FP16) hi part and
    # zero lo part, also after fp16x3's power-of-two scaling; with every
    # partial sum below 2^24 the result is exact.
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
    fastmm.gemm(m, n, k, dev(A), dev(B), C, depth=depth, leaf=1, tile=tile)
    assert np.array_equal(host(C).astype(np.int64), ref)


# (tile, n, depth, bound on the relative Frobenius error)
ERROR_CASES = [(BF, 512, 0, 5e-5), (BF, 1024, 2, 2e-4), (BF, 768, 1, 1e-4),
               (FP, 512, 0, 2e-6), (FP, 1024, 2, 5e-6), (FP, 768, 1, 3e-6), (FP, 1000, 3, 1e-5)]


@pytest.mark.parametrize("dist", ["uniform", "loguniform"])
@pytest.mark.parametrize("tile,n,depth,bound", ERROR_CASES)
def test_split_error_vs_oracle(fastmm, dist, tile, n, depth, bound):
    gen = synthgen.uniform_pm1 if dist == "uniform" else synthgen.loguniform
    A = gen(1001 + 4, n, n)
    B = gen(2001 + 4, n, n)
    C = empty_dev(n, n)
    fastmm.gemm(n, n, n, dev(A), dev(B), C, depth=depth, leaf=1, tile=tile)
    ref = classic.gemm(A, B)
    e = checks.rel_frob(host(C), ref)
    # the FP32 leaf on the same inputs, for the record
    C32 = empty_dev(n, n)
    fastmm.gemm(n, n, n, dev(A), dev(B), C32, depth=depth, leaf=1, tile=0)
    e32 = checks.rel_frob(host(C32), ref)
    say(f"  tile {tile} {dist} n={n} depth={depth}: rel_frob={e:.3e} (fp32 leaf {e32:.3e})")
    assert e <= bound
    if tile == FP:  # FP32-level: within a small factor of the FP32 leaf
        assert e <= 2 * e32


@pytest.mark.parametrize("tile,bound", [(BF, 2e-4), (FP, 2e-5)])
@pytest.mark.parametrize("n", [8192, 16384])
def test_split_depth2_sampled(fastmm, n, tile, bound):
    # n = 8192 and 16384, depth 2, both input distributions.
    rows = synthgen.row_sample(7008, n, 12)
    x = synthgen.signs_pm1(7009, n)
    for dist, gen in [("uniform", synthgen.uniform_pm1), ("loguniform", synthgen.loguniform)]:
        A = gen(1001 + 4, n, n)
        B = gen(2001 + 4, n, n)
        dA, dB, C = dev(A), dev(B), empty_dev(n, n)
        fastmm.gemm(n, n, n, dA, dB, C, depth=2, leaf=1, tile=tile)
        got = host(C)
        e_rows = checks.sampled_rows_rel(got, A, B, rows)
        e_fv = checks.freivalds_rel(got, A, B, x)
        say(f"  tile {tile} {dist} n={n}: sampled-rows rel={e_rows:.3e} freivalds rel={e_fv:.3e}")
        assert e_rows <= bound and e_fv <= bound
        if tile == FP:  # FP32-level: within a small factor of the FP32 leaf
            fastmm.gemm(n, n, n, dA, dB, C, depth=2, leaf=1, tile=0)
            e32 = checks.sampled_rows_rel(host(C), A, B, rows)
            say(f"    fp32 leaf sampled-rows rel={e32:.3e}")
            assert e_rows <= 2 * e32
        del dA, dB, C


def _pow2_scaled(X, row_exp=None, col_exp=None):
    Y = X.astype(np.float64)
    if row_exp is not None:
        Y = np.ldexp(Y, row_exp[:, None])
    if col_exp is not None:
        Y = np.ldexp(Y, col_exp[None, :])
    return Y.astype(np.float32)


@pytest.mark.parametrize("m,k,n", [(300, 200, 257), (129, 515, 640)])
def test_fp16x3_row_column_scaling_is_exact(fastmm, m, k, n):
    # Depth 0: a leaf's scales follow its operands' rows and columns, so
    # scaling row i of A by 2^r_i and column j of B by 2^c_j scales C[i, j] by
    # exactly 2^(r_i + c_j), bit for bit.
    A, B = uniform(3501, m, k), uniform(3502, k, n)
    r = synthgen.int_range(3503, m, 1, -40, 40)[:, 0].astype(np.int64)
    c = synthgen.int_range(3504, 1, n, -30, 30)[0].astype(np.int64)
    C1, C2 = empty_dev(m, n), empty_dev(m, n)
    fastmm.gemm(m, n, k, dev(A), dev(B), C1, depth=0, tile=FP)
    fastmm.gemm(m, n, k, dev(_pow2_scaled(A, row_exp=r)), dev(_pow2_scaled(B, col_exp=c)), C2,
                depth=0, tile=FP)
    assert np.array_equal(host(C2), _pow2_scaled(host(C1), row_exp=r, col_exp=c))


@pytest.mark.parametrize("depth", [1, 2])
def test_fp16x3_global_scaling_is_exact(fastmm, depth):
    # Any depth: a power of two on all of A (B) passes exactly through the
    # FP32 quadrant additions and the per-row (per-column) scales.
    n = 1100
    A, B = uniform(3511, n, n), uniform(3512, n, n)
    C1, C2 = empty_dev(n, n), empty_dev(n, n)
    fastmm.gemm(n, n, n, dev(A), dev(B), C1, depth=depth, leaf=1, tile=FP)
    fastmm.gemm(n, n, n, dev(np.ldexp(A, 60)), dev(np.ldexp(B, -70)), C2, depth=depth, leaf=1,
                tile=FP)
    assert np.array_equal(host(C2), np.ldexp(host(C1), -10))


@pytest.mark.parametrize("depth,row_spread", [(0, 20), (2, 0)])
def test_fp16x3_outside_fp16_range(fastmm, depth, row_spread):
    # Magnitudes near 1e30 and 1e-25, far outside FP16's 6e-8..65504.  At
    # depth 0 the rows of A also differ by up to 2^+-20 and every row is
    # checked on its own.  (Deeper, the quadrant additions mix rows of
    # different magnitude, which costs the small rows accuracy in any
    # arithmetic, FP32 included: there the whole matrix is checked.)
    m, k, n = 640, 700, 520
    r = synthgen.int_range(3521, m, 1, -row_spread, row_spread)[:, 0].astype(np.int64)
    A = _pow2_scaled(uniform(3522, m, k) * np.float32(1e30), row_exp=r)
    B = uniform(3523, k, n) * np.float32(1e-25)
    C = empty_dev(m, n)
    fastmm.gemm(m, n, k, dev(A), dev(B), C, depth=depth, leaf=1, tile=FP)
    got = host(C)
    ref = classic.gemm(A, B)
    e_row = np.max(np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1))
    e = checks.rel_frob(got, ref)
    say(f"  fp16x3 outside FP16 range, depth {depth}: max row rel={e_row:.3e} rel_frob={e:.3e}")
    assert np.isfinite(got).all() and e <= 3e-6
    if depth == 0:
        assert e_row <= 2e-6


def test_fp16x3_host_operands(fastmm):
    # Pinned host operands: the transfer-pipelined path with the FP16 leaf.
    import torch
    m, k, n = 1000, 900, 1100
    A, B = uniform(3531, m, k), uniform(3532, k, n)
    Ah, Bh = torch.from_numpy(A).pin_memory(), torch.from_numpy(B).pin_memory()
    Ch = torch.full((m, n), float("nan")).pin_memory()
    fastmm.gemm(m, n, k, Ah, Bh, Ch, depth=2, leaf=1, tile=FP)
    e = checks.rel_frob(Ch.numpy(), classic.gemm(A, B))
    say(f"  fp16x3 host operands: rel_frob={e:.3e}")
    assert e <= 2e-6


@pytest.mark.parametrize("tile", [BF, FP])
@pytest.mark.parametrize("m,k,n,depth", [(1024, 1024, 1024, 1), (1000, 900, 1100, 2), (700, 645, 1021, 3),
                                         (2048, 1536, 1792, 2)])
def test_split_fused_pack_matches_two_passes(fastmm, monkeypatch, m, k, n, depth, tile):
    # Split-precision leaves at depth >= 1: the last level's pre-additions and
    # the pack pass (for FP16 also the scale pass) run fused, straight from
    # the parent quadrants; they form the same FP32 sums as the pre-addition
    # kernel and the same maxima, so the result equals the separate passes'
    # bit for bit.
    A, B = uniform(3601 + m, m, k), uniform(3602 + n, k, n)
    if tile == FP:  # rows and columns of very different magnitude exercise the scales
        A = _pow2_scaled(A, row_exp=synthgen.int_range(3603, m, 1, -30, 30)[:, 0].astype(np.int64))
        B = _pow2_scaled(B, col_exp=synthgen.int_range(3604, 1, n, -30, 30)[0].astype(np.int64))
    dA, dB = dev(A), dev(B)
    C1, C2 = empty_dev(m, n), empty_dev(m, n)
    # one level of additions per launch, so that the launch counts compare
    # the pack passes alone
    monkeypatch.setenv("FASTMM_TREE_ADDS", "1")
    monkeypatch.delenv("FASTMM_FUSED_PACK", raising=False)
    fastmm.gemm(m, n, k, dA, dB, C1, depth=depth, leaf=1, tile=tile)
    fused_launches = fastmm.get_stats()["launches"]
    monkeypatch.setenv("FASTMM_FUSED_PACK", "0")
    fastmm.gemm(m, n, k, dA, dB, C2, depth=depth, leaf=1, tile=tile)
    two_pass_launches = fastmm.get_stats()["launches"]
    say(f"  fused pack tile {tile} {m}x{k}x{n} depth {depth}: launches {fused_launches} vs {two_pass_launches}")
    assert np.array_equal(host(C1), host(C2))
    if tile == BF:
        assert fused_launches < two_pass_launches
    assert np.isfinite(host(C1)).all()
    if tile == BF:
        assert checks.rel_frob(host(C1), classic.gemm(A, B)) <= 2e-4


@pytest.mark.parametrize("tile", [BF, FP])
def test_split_depth_first_fallback_bitwise(fastmm, monkeypatch, tile):
    # A workspace cap below the level-wise need (packed operands and scale
    # exponents included): the top level runs depth first, each sub-product
    # with its own fused last level; same tree and arithmetic, so the result
    # is bit for bit the level-wise one.
    import torch
    n, depth = 1024, 3
    A, B = dev(uniform(3701, n, n)), dev(uniform(3702, n, n))
    C0 = empty_dev(n, n)
    monkeypatch.delenv("FASTMM_WORKSPACE_LIMIT", raising=False)
    fastmm.gemm(n, n, n, A, B, C0, depth=depth, leaf=1, tile=tile)
    ref = host(C0)
    bfs = fastmm.get_stats()["launches"]
    done = 0
    for limit in [120_000_000, 80_000_000, 60_000_000, 45_000_000]:
        monkeypatch.setenv("FASTMM_WORKSPACE_LIMIT", str(limit))
        C = torch.full((n, n), 7.0, device="cuda")
        rc = fastmm.gemm_raw(n, n, n, A.data_ptr(), n, B.data_ptr(), n, C.data_ptr(), n, depth, 1, tile)
        if rc == fastmm.ERROR_OUT_OF_MEMORY:
            assert torch.all(C == 7.0).item()
            break
        assert rc == fastmm.SUCCESS, fastmm.last_error()
        st = fastmm.get_stats()
        say(f"  tile {tile} limit {limit}: launches {st['launches']} (level-wise {bfs})")
        assert np.array_equal(host(C), ref)
        if st["launches"] > bfs:
            done += 1
    assert done >= 1


def _engine_split(x, d):
    # The library's split of an extent x with d levels left (the leaf extent
    # ceil(x / 2^d), rounded up to a multiple of 4 from 64 on and of 2 from 32
    # on below the top, times 2^(d-1)), restated from its documentation.
    leaf = -(-x // 2 ** d)
    g = 4 if leaf >= 64 else (2 if d >= 2 and leaf >= 32 else 1)
    return (-(-leaf // g) * g) << (d - 1)


def _splits_follow_eq1(x, depth):
    # True when every level of the library's recursion splits x where
    # equation (1) does (at ceil(x / 2)), so that the oracle's emulation and
    # the library take the same quadrants.
    for d in range(depth, 0, -1):
        h = (x + 1) // 2
        if _engine_split(x, d) != h:
            return False
        x = h
    return True


EMU_SHAPES = [(512, 512, 512, 0), (768, 768, 768, 1), (512, 512, 512, 2), (640, 896, 384, 1)]


@pytest.mark.parametrize("tile", [BF, FP])
@pytest.mark.parametrize("dist", ["uniform", "loguniform"])
@pytest.mark.parametrize("m,k,n,depth", EMU_SHAPES)
def test_split_matches_oracle_emulation(fastmm, tile, dist, m, k, n, depth):
    # Against the oracle's emulation of the same arithmetic (hi/lo splits,
    # three products summed in FP64 per leaf, FP32 additions): only the
    # leaves' FP32 accumulation order differs, so the gap is far below each
    # form's own error against the exact product -- a dropped term, a wrong
    # rounding or a wrong scale would show.  Sizes whose halves are
    # multiples of 4, where the engine splits exactly at ceil(m/2).
    # The comparison is only meaningful where the two splits agree.
    assert all(_splits_follow_eq1(x, depth) for x in (m, k, n)), (m, k, n, depth)
    gen = synthgen.uniform_pm1 if dist == "uniform" else synthgen.loguniform
    A, B = gen(3801 + m, m, k), gen(3802 + n, k, n)
    C = empty_dev(m, n)
    fastmm.gemm(m, n, k, dev(A), dev(B), C, depth=depth, leaf=1, tile=tile)
    got = host(C)
    emu = split.winograd_split(A, B, depth, "bf16x3" if tile == BF else "fp16x3")
    exact = classic.gemm(A, B)
    e_emu = checks.rel_frob(got, emu)
    e_exact = checks.rel_frob(got, exact)
    say(f"  tile {tile} {dist} {m}x{k}x{n} d{depth}: vs emulation {e_emu:.2e}, vs exact {e_exact:.2e}")
    assert e_emu <= 1.5e-6  # measured 2.3e-7 (depth 0) to 9.1e-7 (depth 2)
    if tile == BF:
        assert e_emu <= 0.25 * e_exact  # measured 0.03-0.06 of it

