"""ORACLE (test infrastructure): the classic product c_ij = sum_k a_ik b_kj.

Equation (6) of Section 3.3 defines every entry of the result as a
row-by-column sum; the Winograd recursion reaches the same matrix with fewer
products, so this definition is the oracle for every depth.  The heavy loops
are in ``ref_gemm.c`` (plain triple loop, FP64 or int64 accumulation,
ascending k per entry); ``brute_force`` is a pure-Python triple loop used to
pin the C loops on tiny inputs.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import LIB_PATH, build

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        i64, vp = ctypes.c_int64, ctypes.c_void_p
        lib.ref_gemm_f64.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64]
        lib.ref_gemm_f32in.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64]
        lib.ref_gemm_rows_f32in.argtypes = [i64, vp, i64, i64, vp, i64, vp, i64, vp]
        lib.ref_gemv_f32in.argtypes = [i64, i64, vp, i64, vp, vp]
        lib.ref_gemm_i64.argtypes = [i64, i64, i64, vp, i64, vp, i64, vp, i64]
        lib.ref_num_threads.argtypes = []
        lib.ref_num_threads.restype = ctypes.c_int
        for name in ("ref_gemm_f64", "ref_gemm_f32in", "ref_gemm_rows_f32in",
                     "ref_gemv_f32in", "ref_gemm_i64"):
            getattr(lib, name).restype = None
        _lib = lib
    return _lib


def num_threads() -> int:
    """OpenMP threads the C loops use (OMP_NUM_THREADS, else all cores)."""
    return int(_load().ref_num_threads())


def _rowmajor(x: np.ndarray, dtype) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=dtype)


def gemm(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """C = A B with FP64 accumulation.  FP32 inputs are widened exactly; the
    result is float64.  int64 inputs give an exact int64 result."""
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("shape mismatch")
    M, K = A.shape
    N = B.shape[1]
    lib = _load()
    if A.dtype == np.int64 and B.dtype == np.int64:
        A = _rowmajor(A, np.int64)
        B = _rowmajor(B, np.int64)
        C = np.empty((M, N), dtype=np.int64)
        if M and N:
            lib.ref_gemm_i64(M, N, K, A.ctypes.data, max(K, 1), B.ctypes.data, max(N, 1),
                             C.ctypes.data, N)
        return C
    if A.dtype == np.float32 and B.dtype == np.float32:
        A = _rowmajor(A, np.float32)
        B = _rowmajor(B, np.float32)
        C = np.empty((M, N), dtype=np.float64)
        if M and N:
            lib.ref_gemm_f32in(M, N, K, A.ctypes.data, max(K, 1), B.ctypes.data, max(N, 1),
                               C.ctypes.data, N)
        return C
    A = _rowmajor(A, np.float64)
    B = _rowmajor(B, np.float64)
    C = np.empty((M, N), dtype=np.float64)
    if M and N:
        lib.ref_gemm_f64(M, N, K, A.ctypes.data, max(K, 1), B.ctypes.data, max(N, 1),
                         C.ctypes.data, N)
    return C


def gemm_rows(A: np.ndarray, B: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """Rows ``rows`` of A B (FP32 inputs, FP64 accumulation), for problems
    whose full product the CPU cannot afford on every check."""
    A = _rowmajor(A, np.float32)
    B = _rowmajor(B, np.float32)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= A.shape[0]):
        raise ValueError("row index out of range")
    K = A.shape[1]
    N = B.shape[1]
    out = np.empty((rows.size, N), dtype=np.float64)
    if rows.size and N:
        _load().ref_gemm_rows_f32in(rows.size, rows.ctypes.data, N, K, A.ctypes.data,
                                    max(K, 1), B.ctypes.data, max(N, 1), out.ctypes.data)
    return out


def gemv(X: np.ndarray, v: np.ndarray) -> np.ndarray:
    """y = X v with X FP32 (widened) and v FP64, FP64 accumulation."""
    X = _rowmajor(X, np.float32)
    v = np.ascontiguousarray(v, dtype=np.float64)
    M, N = X.shape
    y = np.empty(M, dtype=np.float64)
    if M:
        _load().ref_gemv_f32in(M, N, X.ctypes.data, max(N, 1), v.ctypes.data, y.ctypes.data)
    return y


def brute_force(A, B):
    """Pure-Python triple loop over nested lists / arrays, for n <= ~32.
    Exact for Python ints; float inputs accumulate in Python floats (FP64)."""
    M = len(A)
    K = len(A[0]) if M else 0
    N = len(B[0]) if len(B) else 0
    C = [[0 for _ in range(N)] for _ in range(M)]
    for i in range(M):
        for j in range(N):
            s = 0
            for k in range(K):
                s += A[i][k] * B[k][j]
            C[i][j] = s
    return C
