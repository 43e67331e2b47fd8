"""Pins of the oracle's split-precision emulation (oracle/split.py): BF16
rounding against hand-worked bit patterns (ties to even), the split residual
bounds that follow from 8- and 11-bit significands, the scaling rule, exact
products on integers the splits hold exactly, error bounds on random inputs,
and exact power-of-two equivariance of the scaled FP16 form."""
import numpy as np
import pytest

import synthgen
from oracle import classic, split
from oracle import winograd as W


def test_bf16_round_ties_to_even():
    x = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, -(1 + 2**-8), 1 + 2**-8 + 2**-20, 3.0, 0.0],
                 dtype=np.float32)
    want = np.array([1.0, 1.0, 1 + 2**-6, -1.0, 1 + 2**-7, 3.0, 0.0], dtype=np.float32)
    assert np.array_equal(split.bf16_round(x), want)
    # the result keeps only the top 16 bits
    y = split.bf16_round(synthgen.uniform_pm1(11, 64, 64))
    assert np.all((y.view(np.uint32) & 0xFFFF) == 0)


def test_split_residual_bounds():
    x = synthgen.loguniform(12, 128, 128)
    hi, lo = split.split_bf16(x)
    assert np.all(np.abs(x.astype(np.float64) - hi - lo) <= 2.0**-17 * np.abs(x))
    assert np.all(np.abs(lo) <= 2.0**-8 * np.abs(x))
    y = (np.abs(synthgen.uniform_pm1(13, 128, 128)) * 2**15).astype(np.float32) + np.float32(0.125)
    hi16, lo16 = split.split_fp16(y)
    assert np.all(np.abs(y.astype(np.float64) - hi16 - lo16) <= 2.0**-22 * np.abs(y))


def test_scale_exponents_rule():
    m = np.abs(synthgen.loguniform(14, 1, 4096)[0]).astype(np.float64)
    e = split.scale_exponents(m)
    s = np.ldexp(m, -e)
    assert np.all((s >= 2**14) & (s < 2**15))
    assert split.scale_exponents(np.array([0.0]))[0] == 0
    assert split.scale_exponents(np.array([2.0**15]))[0] == 1


@pytest.mark.parametrize("form,lim", [("bf16x3", 256), ("fp16x3", 2048)])
def test_leaf_exact_on_representable_integers(form, lim):
    a = synthgen.int_range(15, 40, 70, -lim, lim)
    b = synthgen.int_range(16, 70, 30, -3, 3)
    leaf = split.leaf_bf16x3 if form == "bf16x3" else split.leaf_fp16x3
    got = leaf(a, b)
    assert np.array_equal(got.astype(np.int64), classic.gemm(a.astype(np.int64), b.astype(np.int64)))


@pytest.mark.parametrize("form,bound", [("bf16x3", 2.0**-14), ("fp16x3", 2.0**-19)])
def test_leaf_error_on_random_inputs(form, bound):
    # the dropped lo*lo term and the split residuals are at most a few units
    # of 2^-16 (BF16) or 2^-22 (FP16) of each product term
    a = synthgen.uniform_pm1(17, 96, 200)
    b = synthgen.loguniform(18, 200, 80)
    leaf = split.leaf_bf16x3 if form == "bf16x3" else split.leaf_fp16x3
    ref = classic.gemm(a, b)
    e = np.abs(leaf(a, b).astype(np.float64) - ref)
    scale = np.abs(a).astype(np.float64) @ np.abs(b).astype(np.float64)
    assert np.all(e <= bound * scale)


def test_fp16_scaling_is_exact():
    a = synthgen.uniform_pm1(19, 50, 64)
    b = synthgen.uniform_pm1(20, 64, 40)
    r = synthgen.int_range(21, 50, 1, -30, 30)[:, 0].astype(np.int64)
    c = synthgen.int_range(22, 1, 40, -30, 30)[0].astype(np.int64)
    a2 = np.ldexp(a, r[:, None]).astype(np.float32)
    b2 = np.ldexp(b, c[None, :]).astype(np.float32)
    got = split.leaf_fp16x3(a2, b2)
    want = np.ldexp(split.leaf_fp16x3(a, b), r[:, None] + c[None, :]).astype(np.float32)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("form", ["bf16x3", "fp16x3"])
def test_winograd_split_exact_on_small_integers(form):
    a = synthgen.int_range(23, 60, 44, -2, 2)
    b = synthgen.int_range(24, 44, 52, -2, 2)
    cert = W.Certificate()
    ref = W.winograd(a.astype(np.int64), b.astype(np.int64), 2, 1, cert)
    assert cert.exact_in_fp32
    got = split.winograd_split(a, b, 2, form)
    assert np.array_equal(got.astype(np.int64), ref)
