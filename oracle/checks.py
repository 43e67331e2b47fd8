"""ORACLE (test infrastructure): error measures and probabilistic checks.

The paper reports no numerical analysis (Section 1 states that none is
given), so tolerances are stated in the tests, against these measures.
"""
from __future__ import annotations

import numpy as np

from . import classic


def rel_frob(C: np.ndarray, ref: np.ndarray) -> float:
    """||C - ref||_F / ||ref||_F, computed in FP64."""
    C = np.asarray(C, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    num = np.linalg.norm(C - ref)
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return float(num / den)


def sampled_rows_rel(C: np.ndarray, A: np.ndarray, B: np.ndarray, rows: np.ndarray) -> float:
    """Relative Frobenius error of the selected rows of C against the exact
    (FP64-accumulated) rows of A B: an unbiased sample of the full error."""
    ref = classic.gemm_rows(A, B, rows)
    return rel_frob(np.asarray(C)[rows], ref)


def freivalds_rel(C: np.ndarray, A: np.ndarray, B: np.ndarray, x: np.ndarray) -> float:
    """Freivalds' check: ||C x - A (B x)|| / ||A (B x)|| for a +-1 vector x.
    A wrong or missing block of C makes this O(1) with high probability; a
    correct FP32 result gives about the relative Frobenius error."""
    Bx = classic.gemv(B, x)
    ABx = classic.gemv(A, Bx)
    Cx = classic.gemv(C, x)
    den = np.linalg.norm(ABx)
    return float(np.linalg.norm(Cx - ABx) / den) if den else float(np.linalg.norm(Cx))
