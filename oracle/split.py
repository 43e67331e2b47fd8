"""ORACLE (test infrastructure): the precision forms of the leaf product,
emulated on the CPU.

These forms are not in the paper (its leaves are FP32); they reproduce, in
plain numpy, what the library's split-precision leaves are defined to
compute, so that the GPU results can be compared with their own arithmetic
and not only with the exact product:

* split BF16: x = hi + lo with hi = bf16(x) and lo = bf16(x - hi), each
  rounded to nearest even (the BF16 format keeps the top 16 bits of an FP32
  number); a*b taken as hi_a hi_b + hi_a lo_b + lo_a hi_b;
* scaled split FP16: every row r of the left operand and every column c of
  the right one is multiplied by 2^-e, e = exponent that brings the row's
  (column's) largest magnitude into [2^14, 2^15) (e = 0 for a zero row), then
  split into hi + lo FP16 (numpy's float32 -> float16 conversion rounds to
  nearest even) and the sum scaled back by 2^(e_r + e_c).

The three partial products are summed in FP64 and the leaf result rounded
once to FP32.  ``winograd_split`` runs the recursion with FP32 additions (the
chains of ``winograd.preadd_a/b`` and ``postadd_full`` on float32 arrays) and
these leaves; it splits quadrants at ceil(m/2) (equation (1)), so compare it
with the GPU only at sizes whose halves are multiples of 4.
"""
from __future__ import annotations

import numpy as np

from . import winograd as W


def bf16_round(x: np.ndarray) -> np.ndarray:
    """float32 values rounded to BF16 (nearest, ties to even), as float32."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def split_bf16(x: np.ndarray):
    """(hi, lo) as float32 arrays holding BF16 values; x - hi is exact in FP32."""
    x = np.asarray(x, dtype=np.float32)
    hi = bf16_round(x)
    lo = bf16_round(x - hi)
    return hi, lo


def scale_exponents(m: np.ndarray) -> np.ndarray:
    """e with m * 2^-e in [2^14, 2^15) for each maximum m; 0 for m = 0."""
    m = np.asarray(m, dtype=np.float64)
    _, e = np.frexp(m)  # m = f * 2^e, f in [0.5, 1)
    e = e.astype(np.int64) - 15
    return np.where(m > 0, e, 0)


def split_fp16(y: np.ndarray):
    """(hi, lo) as float32 arrays holding FP16 values of already scaled y."""
    y = np.asarray(y, dtype=np.float32)
    hi = y.astype(np.float16).astype(np.float32)
    lo = (y - hi).astype(np.float16).astype(np.float32)
    return hi, lo


def _three_products(ha, la, hb, lb) -> np.ndarray:
    ha, la, hb, lb = (v.astype(np.float64) for v in (ha, la, hb, lb))
    return ha @ hb + ha @ lb + la @ hb


def leaf_bf16x3(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """One leaf product in split BF16 (FP64 sum, rounded to FP32)."""
    ha, la = split_bf16(a)
    hb, lb = split_bf16(b)
    return _three_products(ha, la, hb, lb).astype(np.float32)


def leaf_fp16x3(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """One leaf product in scaled split FP16 (FP64 sum, rounded to FP32)."""
    a = np.asarray(a, dtype=np.float32)
    b = np.asarray(b, dtype=np.float32)
    ea = scale_exponents(np.abs(a).max(axis=1, initial=0.0))
    eb = scale_exponents(np.abs(b).max(axis=0, initial=0.0))
    ha, la = split_fp16(np.ldexp(a, -ea[:, None]).astype(np.float32))
    hb, lb = split_fp16(np.ldexp(b, -eb[None, :]).astype(np.float32))
    s = _three_products(ha, la, hb, lb)
    return np.ldexp(s, ea[:, None] + eb[None, :]).astype(np.float32)


def winograd_split(A: np.ndarray, B: np.ndarray, depth: int, form: str) -> np.ndarray:
    """Winograd's recursion (``depth`` levels, equation (1) split) with FP32
    additions and split-precision leaves (form "bf16x3" or "fp16x3")."""
    leaf = {"bf16x3": leaf_bf16x3, "fp16x3": leaf_fp16x3}[form]
    return _rec(np.asarray(A, np.float32), np.asarray(B, np.float32), depth, leaf)


def _rec(A, B, levels, leaf):
    m, k = A.shape
    n = B.shape[1]
    if levels == 0 or min(m, k, n) < 2:
        return leaf(A, B)
    A11, A12, A21, A22 = W.quadrants(A)
    B11, B12, B21, B22 = W.quadrants(B)
    S = W.preadd_a(A11, A12, A21, A22)
    T = W.preadd_b(B11, B12, B21, B22)
    P = [_rec(x, y, levels - 1, leaf) for x, y in W.product_pairs(A11, A12, A22, B11, B21, B22, S, T)]
    C11, C12, C21, C22 = W.postadd_full(*P)[:4]
    return W.assemble(C11, C12, C21, C22, m, n)
