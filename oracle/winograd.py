"""ORACLE (test infrastructure): the recursive algorithms of the paper, on the CPU.

Quadrant split -- equation (1), Section 3.1: any m x n matrix D is cut into
D0 (top-left, ceil(m/2) x ceil(n/2)), D1 (top-right), D2 (bottom-left) and D3
(bottom-right, floor(m/2) x floor(n/2)).  Below, X11, X12, X21, X22 name D0,
D1, D2, D3.  Odd extents are handled by virtual zero padding: every quadrant
is taken as ceil(m/2) x ceil(n/2) with the missing row/column read as zero.
That is Winograd on the zero-padded matrix, so the cropped result is exact.

Winograd's variant of Strassen's recursion.  The paper names it (Section 4.1,
the "SW" curve, and the closing remark of Section 4.3 that a fast recursive
algorithm could replace the classic one at the leaf boundary) but never prints
its formulas.  This file uses the standard schedule of Winograd's variant: 7
products and 15 quadrant additions per level,

    S1 = A21 + A22   S2 = S1 - A11    S3 = A11 - A21   S4 = A12 - S2
    T1 = B12 - B11   T2 = B22 - T1    T3 = B22 - B12   T4 = T2 - B21
    P1 = A11 B11     P2 = A12 B21     P3 = S4 B22      P4 = A22 T4
    P5 = S1 T1       P6 = S2 T2       P7 = S3 T3
    C11 = P1 + P2    U2 = P1 + P6     U3 = U2 + P7     U4 = U2 + P5
    C12 = U4 + P3    C21 = U3 - P4    C22 = U3 + P5

Stop rule (Section 3.1 recursion point; Table 2 leaf): a node (m, k, n) is
split iff levels remain and floor(min(m, k, n) / 2) >= max(leaf, 1).  With
leaf = 3008 this stops exactly below the paper's 6016 recursion point.

The classic 8-product recursion (Table 1, left column ``RMUL``, and the
multiply-add right column) and the two-device column split of equations
(3)-(4) are here too, as further algebraic pins.
"""
from __future__ import annotations

import numpy as np

from . import classic

# --------------------------------------------------------------------------
# Equation (1): quadrant extents and the split rule.


def half_up(m: int) -> int:
    """Extent of quadrant 0 along a dimension of size m (ceil(m/2))."""
    return (m + 1) // 2


def half_down(m: int) -> int:
    """Extent of quadrant 3 along a dimension of size m (floor(m/2))."""
    return m // 2


def splits(m: int, k: int, n: int, levels_left: int, leaf: int) -> bool:
    """Whether node (m, k, n) recurses (stop rule above)."""
    return levels_left > 0 and min(m, k, n) // 2 >= max(int(leaf), 1)


def quadrants(D: np.ndarray):
    """The four quadrants of D per equation (1), each zero-padded to
    ceil(rows/2) x ceil(cols/2).  Returns (D11, D12, D21, D22)."""
    r, c = D.shape
    r2, c2 = half_up(r), half_up(c)
    P = np.zeros((2 * r2, 2 * c2), dtype=D.dtype)
    P[:r, :c] = D
    return P[:r2, :c2], P[:r2, c2:], P[r2:, :c2], P[r2:, c2:]


def assemble(C11, C12, C21, C22, rows: int, cols: int) -> np.ndarray:
    """Inverse of ``quadrants``: place four blocks and crop to rows x cols."""
    top = np.concatenate([C11, C12], axis=1)
    bot = np.concatenate([C21, C22], axis=1)
    return np.concatenate([top, bot], axis=0)[:rows, :cols]


# --------------------------------------------------------------------------
# One level of Winograd's schedule.  The same expressions serve every dtype:
# with float32 arrays each operation rounds to FP32 (IEEE round-to-nearest),
# which makes these the reference for the GPU's fused addition kernels.


def preadd_a(A11, A12, A21, A22):
    """(S1, S2, S3, S4) from the A quadrants."""
    S1 = A21 + A22
    S2 = S1 - A11
    S3 = A11 - A21
    S4 = A12 - S2
    return S1, S2, S3, S4


def preadd_b(B11, B12, B21, B22):
    """(T1, T2, T3, T4) from the B quadrants."""
    T1 = B12 - B11
    T2 = B22 - T1
    T3 = B22 - B12
    T4 = T2 - B21
    return T1, T2, T3, T4


def postadd_full(P1, P2, P3, P4, P5, P6, P7):
    """(C11, C12, C21, C22, U2, U3, U4) from the seven products."""
    C11 = P1 + P2
    U2 = P1 + P6
    U3 = U2 + P7
    U4 = U2 + P5
    C12 = U4 + P3
    C21 = U3 - P4
    C22 = U3 + P5
    return C11, C12, C21, C22, U2, U3, U4


def postadd(P1, P2, P3, P4, P5, P6, P7):
    """(C11, C12, C21, C22) from the seven products."""
    return postadd_full(P1, P2, P3, P4, P5, P6, P7)[:4]


def product_pairs(A11, A12, A22, B11, B21, B22, S, T):
    """The seven (left, right) operand pairs of P1..P7, in order."""
    S1, S2, S3, S4 = S
    T1, T2, T3, T4 = T
    return [(A11, B11), (A12, B21), (S4, B22), (A22, T4), (S1, T1), (S2, T2), (S3, T3)]


# --------------------------------------------------------------------------
# The recursion.


class Certificate:
    """Largest magnitudes met during an integer run.  If every recorded value
    and every leaf's k * max|a| * max|b| stays below 2**24, an FP32
    evaluation of the same schedule performs only exact operations (each
    partial sum is an integer of magnitude < 2**24), so an FP32 GPU result
    must equal the exact product bit for bit."""

    def __init__(self):
        self.max_intermediate = 0
        self.max_leaf_bound = 0
        self.leaves = 0

    def see(self, *arrays):
        for a in arrays:
            if a.size:
                self.max_intermediate = max(self.max_intermediate, int(np.abs(a).max()))

    def see_leaf(self, a, b):
        self.leaves += 1
        k = a.shape[1]
        if a.size and b.size:
            bound = k * int(np.abs(a).max()) * int(np.abs(b).max())
            self.max_leaf_bound = max(self.max_leaf_bound, bound)

    @property
    def exact_in_fp32(self) -> bool:
        return self.max_intermediate < 2**24 and self.max_leaf_bound < 2**24


def _leaf_product(a, b):
    if a.dtype == np.int64:
        return classic.gemm(a, b)
    return classic.gemm(a.astype(np.float64), b.astype(np.float64))


def winograd(A: np.ndarray, B: np.ndarray, depth: int, leaf: int = 1,
             cert: Certificate | None = None, leaf_fn=None) -> np.ndarray:
    """C = A B by Winograd's recursion, at most ``depth`` levels.

    int64 inputs: exact integer arithmetic (the result must equal the
    classic product exactly).  Floating inputs: every step in FP64, leaves
    by the FP64-accumulated triple loop.  ``leaf_fn`` replaces the leaf
    product (used by tests that plant a fault)."""
    if A.dtype != np.int64:
        A = A.astype(np.float64)
        B = B.astype(np.float64)
    return _wino(A, B, depth, leaf, cert, leaf_fn or _leaf_product)


def _wino(A, B, levels, leaf, cert, leaf_fn):
    m, k = A.shape
    n = B.shape[1]
    if not splits(m, k, n, levels, leaf):
        if cert is not None:
            cert.see_leaf(A, B)
        C = leaf_fn(A, B)
        if cert is not None:
            cert.see(C)
        return C
    A11, A12, A21, A22 = quadrants(A)
    B11, B12, B21, B22 = quadrants(B)
    S = preadd_a(A11, A12, A21, A22)
    T = preadd_b(B11, B12, B21, B22)
    if cert is not None:
        cert.see(*S, *T)
    pairs = product_pairs(A11, A12, A22, B11, B21, B22, S, T)
    P = [_wino(x, y, levels - 1, leaf, cert, leaf_fn) for x, y in pairs]
    C11, C12, C21, C22, U2, U3, U4 = postadd_full(*P)
    if cert is not None:
        cert.see(C11, U2, U3, U4, C12, C21, C22)
    return assemble(C11, C12, C21, C22, m, n)


def effective_depth(m: int, k: int, n: int, depth: int, leaf: int) -> int:
    """Levels the stop rule actually takes (all nodes of a level share the
    parent's ceil extents, so one chain of ceil halvings decides)."""
    d = 0
    while splits(m, k, n, depth - d, leaf):
        m, k, n = half_up(m), half_up(k), half_up(n)
        d += 1
    return d


def structure(M: int, N: int, K: int, depth: int, leaf: int) -> dict:
    """Closed-form counts of the recursion (virtual, zero-padded extents).

    Every node of level l has extents (m_l, k_l, n_l) with m_{l+1} =
    ceil(m_l / 2), so there are 7**d leaves of (m_d, k_d, n_d).  Per internal
    node of level l the pre-additions read 4 and write 4 quadrants of each
    operand and the post-additions read 7 and write 4 quadrants of the
    result; 15 quadrant additions in all."""
    d = effective_depth(M, K, N, depth, leaf)
    dims = [(M, K, N)]
    for _ in range(d):
        m, k, n = dims[-1]
        dims.append((half_up(m), half_up(k), half_up(n)))
    mL, kL, nL = dims[-1]
    add_bytes = 0
    add_elems = 0
    levels = []
    for lev in range(d):
        nodes = 7 ** lev
        m2, k2, n2 = dims[lev + 1]
        pre_a = nodes * 32 * m2 * k2
        pre_b = nodes * 32 * k2 * n2
        post = nodes * 44 * m2 * n2
        add_bytes += pre_a + pre_b + post
        add_elems += nodes * (4 * m2 * k2 + 4 * k2 * n2 + 7 * m2 * n2)
        levels.append({"level": lev, "nodes": nodes, "child_dims": (m2, k2, n2),
                       "preadd_a_bytes": pre_a, "preadd_b_bytes": pre_b,
                       "postadd_bytes": post})
    return {
        "depth": d,
        "leaves": 7 ** d,
        "leaf_dims": (mL, kL, nL),
        "leaf_flops": 7 ** d * 2 * mL * nL * kL,
        "add_bytes": add_bytes,
        "add_elements": add_elems,
        "levels": levels,
        "dims": dims,
    }


# --------------------------------------------------------------------------
# Table 1: the classic 8-product recursion (C = AB and C += AB), and the
# two-device split of equations (3)-(4).  Pins for the comparators.


def rmul(A, B, depth: int, leaf: int = 1):
    """Table 1, left column: C0 = A0 B0, C1 = A0 B1, C2 = A2 B0, C3 = A2 B1,
    then C0 += A1 B2, C1 += A1 B3, C2 += A3 B2, C3 += A3 B3 (quadrants as in
    equation (1), D0..D3 = D11, D12, D21, D22)."""
    m, k = A.shape
    n = B.shape[1]
    C = np.zeros((m, n), dtype=np.result_type(A.dtype, B.dtype, np.float64)
                 if A.dtype != np.int64 else np.int64)
    rmul_add(C, A, B, depth, leaf, overwrite=True)
    return C


def rmul_add(C, A, B, depth: int, leaf: int = 1, overwrite: bool = False):
    """Table 1, right column (C += AB); with ``overwrite`` the first product
    of each quadrant assigns, as in the left column."""
    m, k = A.shape
    n = B.shape[1]
    if not splits(m, k, n, depth, leaf):
        P = _leaf_product(A, B)
        if overwrite:
            C[...] = P
        else:
            C += P
        return
    A0, A1, A2, A3 = quadrants(A)
    B0, B1, B2, B3 = quadrants(B)
    m2, n2 = half_up(m), half_up(n)
    Cp = np.zeros((2 * m2, 2 * n2), dtype=C.dtype)
    Cp[:m, :n] = C
    C0, C1, C2, C3 = Cp[:m2, :n2], Cp[:m2, n2:], Cp[m2:, :n2], Cp[m2:, n2:]
    rmul_add(C0, A0, B0, depth - 1, leaf, overwrite)
    rmul_add(C1, A0, B1, depth - 1, leaf, overwrite)
    rmul_add(C2, A2, B0, depth - 1, leaf, overwrite)
    rmul_add(C3, A2, B1, depth - 1, leaf, overwrite)
    rmul_add(C0, A1, B2, depth - 1, leaf)
    rmul_add(C1, A1, B3, depth - 1, leaf)
    rmul_add(C2, A3, B2, depth - 1, leaf)
    rmul_add(C3, A3, B3, depth - 1, leaf)
    C[...] = Cp[:m, :n]


def two_device_split(A, B):
    """Equations (3)-(4): device 0 computes C0 and C2 (the left column of
    quadrants, from B0 and B2), device 1 computes C1 and C3.  Returns the two
    column panels (left, right) of C = AB, each by its own four products."""
    m = A.shape[0]
    n = B.shape[1]
    A0, A1, A2, A3 = quadrants(A)
    B0, B1, B2, B3 = quadrants(B)
    g = _leaf_product
    C0 = g(A0, B0) + g(A1, B2)
    C2 = g(A2, B0) + g(A3, B2)
    C1 = g(A0, B1) + g(A1, B3)
    C3 = g(A2, B1) + g(A3, B3)
    left = np.concatenate([C0, C2], axis=0)[:m]
    right = np.concatenate([C1, C3], axis=0)[:m, : n - half_up(n)]
    return left, right
