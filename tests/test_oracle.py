"""Pins for the CPU oracle: each checks it against something other than
itself (hand-worked values, closed forms, brute force, exact integer
identities), chosen so that a dropped term, a wrong sign or index or a
transposed operand fails at least one of them."""
import json
import os

import numpy as np
import pytest

import synthgen
from oracle import checks, classic, mlp
from oracle import winograd as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ints(seed, r, c, lo=-3, hi=3):
    return synthgen.int_range_np(seed, r, c, lo, hi).astype(np.int64)


# ---------------------------------------------------------------- classic

@pytest.mark.parametrize("m,k,n", [(1, 1, 1), (3, 5, 2), (7, 4, 9), (16, 16, 16), (5, 1, 6)])
def test_classic_matches_brute_force(m, k, n):
    A = ints(11 + m, m, k)
    B = ints(12 + n, k, n)
    ref = np.array(classic.brute_force(A.tolist(), B.tolist()), dtype=np.int64)
    assert np.array_equal(classic.gemm(A, B), ref)
    Af = synthgen.uniform_pm1_np(21, m, k)
    Bf = synthgen.uniform_pm1_np(22, k, n)
    bf = np.array(classic.brute_force(Af.astype(float).tolist(), Bf.astype(float).tolist()))
    np.testing.assert_allclose(classic.gemm(Af, Bf), bf, rtol=0, atol=1e-14)


def test_classic_closed_form_polynomial():
    # a_ik = i + k, b_kj = k - j  =>  c_ij = i*S1 - i*j*K + S2 - j*S1
    # with S1 = sum k = K(K-1)/2 and S2 = sum k^2 = (K-1)K(2K-1)/6.
    M, K, N = 13, 17, 11
    i = np.arange(M)[:, None]
    j = np.arange(N)[None, :]
    kk = np.arange(K)
    A = (np.arange(M)[:, None] + kk[None, :]).astype(np.int64)
    B = (kk[:, None] - np.arange(N)[None, :]).astype(np.int64)
    S1 = K * (K - 1) // 2
    S2 = (K - 1) * K * (2 * K - 1) // 6
    expect = i * S1 - i * j * K + S2 - j * S1
    assert np.array_equal(classic.gemm(A, B), expect)
    assert np.array_equal(classic.gemm(A.astype(np.float32), B.astype(np.float32)), expect)


def test_classic_identity_and_ones():
    A = synthgen.uniform_pm1_np(5, 40, 33)
    I = np.eye(33, dtype=np.float32)
    assert np.array_equal(classic.gemm(A, I), A.astype(np.float64))
    ones_a = np.ones((9, 23), np.float32)
    ones_b = np.ones((23, 4), np.float32)
    assert np.all(classic.gemm(ones_a, ones_b) == 23.0)


def test_classic_not_transposed():
    # A non-square, non-symmetric case where A B and B^T A^T-style slips differ.
    A = np.array([[1, 2, 3]], dtype=np.int64)
    B = np.array([[1], [10], [100]], dtype=np.int64)
    assert classic.gemm(A, B).tolist() == [[321]]
    assert classic.gemm(B, A).tolist() == [[1, 2, 3], [10, 20, 30], [100, 200, 300]]


def test_classic_empty_k_gives_zero():
    A = np.zeros((3, 0), np.float32)
    B = np.zeros((0, 4), np.float32)
    assert np.array_equal(classic.gemm(A, B), np.zeros((3, 4)))


def test_gemm_rows_and_gemv():
    A = synthgen.uniform_pm1_np(7, 50, 30)
    B = synthgen.uniform_pm1_np(8, 30, 20)
    full = classic.gemm(A, B)
    rows = np.array([0, 3, 49])
    assert np.array_equal(classic.gemm_rows(A, B, rows), full[rows])
    x = synthgen.signs_pm1(9, 20)
    np.testing.assert_allclose(classic.gemv(full.astype(np.float32), x),
                               full.astype(np.float32).astype(np.float64) @ x, rtol=1e-13)


# ---------------------------------------------------------------- quadrants (eq. 1)

@pytest.mark.parametrize("r,c", [(4, 6), (5, 7), (1, 3), (2, 1)])
def test_quadrant_extents_equation_1(r, c):
    D = np.arange(1, r * c + 1, dtype=np.int64).reshape(r, c)
    D11, D12, D21, D22 = W.quadrants(D)
    r0, c0 = (r + 1) // 2, (c + 1) // 2
    for q in (D11, D12, D21, D22):
        assert q.shape == (r0, c0)
    # D0 is ceil x ceil and fully populated; D3 holds floor x floor values.
    assert np.all(D11 != 0)
    assert np.count_nonzero(D22) == (r // 2) * (c // 2)
    assert np.array_equal(W.assemble(D11, D12, D21, D22, r, c), D)


# ---------------------------------------------------------------- Winograd

def test_winograd_hand_worked_2x2():
    with open(os.path.join(GOLDEN, "winograd_2x2_by_hand.json")) as f:
        g = json.load(f)
    A = np.array(g["A"], dtype=np.int64)
    B = np.array(g["B"], dtype=np.int64)
    A11, A12, A21, A22 = W.quadrants(A)
    B11, B12, B21, B22 = W.quadrants(B)
    S = W.preadd_a(A11, A12, A21, A22)
    T = W.preadd_b(B11, B12, B21, B22)
    assert [int(x[0, 0]) for x in S] == [g["S"][f"S{i}"] for i in range(1, 5)]
    assert [int(x[0, 0]) for x in T] == [g["T"][f"T{i}"] for i in range(1, 5)]
    pairs = W.product_pairs(A11, A12, A22, B11, B21, B22, S, T)
    P = [x @ y for x, y in pairs]
    assert [int(p[0, 0]) for p in P] == [g["P"][f"P{i}"] for i in range(1, 8)]
    C11, C12, C21, C22, U2, U3, U4 = W.postadd_full(*P)
    assert [int(U2[0, 0]), int(U3[0, 0]), int(U4[0, 0])] == [g["U"]["U2"], g["U"]["U3"], g["U"]["U4"]]
    assert W.winograd(A, B, 1).tolist() == g["C"]


SHAPES = [(8, 8, 8), (16, 12, 20), (13, 7, 11), (33, 31, 35), (64, 64, 64), (5, 40, 3),
          (1, 9, 1), (2, 2, 2), (17, 1, 5)]


@pytest.mark.parametrize("m,k,n", SHAPES)
@pytest.mark.parametrize("depth", [0, 1, 2, 3, 4])
def test_winograd_int64_equals_classic_exactly(m, k, n, depth):
    A = ints(100 + m, m, k)
    B = ints(200 + n, k, n)
    assert np.array_equal(W.winograd(A, B, depth, 1), classic.gemm(A, B))


@pytest.mark.parametrize("leaf", [1, 2, 3, 8])
def test_winograd_leaf_cutoff_int64(leaf):
    A = ints(301, 37, 30)
    B = ints(302, 30, 45)
    cert = W.Certificate()
    C = W.winograd(A, B, 6, leaf, cert)
    assert np.array_equal(C, classic.gemm(A, B))
    assert cert.leaves == 7 ** W.effective_depth(37, 30, 45, 6, leaf)


def test_winograd_fp64_close_to_classic():
    A = synthgen.uniform_pm1_np(1001, 96, 80)
    B = synthgen.uniform_pm1_np(2001, 80, 72)
    ref = classic.gemm(A, B)
    for d in range(4):
        assert checks.rel_frob(W.winograd(A, B, d, 1), ref) < 1e-12


def test_winograd_all_ones_equals_k():
    for (m, k, n), d in [((32, 24, 16), 3), ((19, 23, 17), 3), ((64, 64, 64), 4)]:
        C = W.winograd(np.ones((m, k), np.float32), np.ones((k, n), np.float32), d, 1)
        assert np.all(C == k)


def test_winograd_fp32_adds_bitwise_chain():
    # FP32 evaluation: each step is one IEEE FP32 operation; check S2 equals
    # the rounded FP32 value of (rounded S1) - A11, not the exact one.
    a21 = np.float32(1.0)
    a22 = np.float32(2.0 ** -24)
    a11 = np.float32(1.0)
    S1, S2, S3, S4 = W.preadd_a(np.array([a11]), np.array([np.float32(0)]),
                                np.array([a21]), np.array([a22]))
    assert S1.dtype == np.float32 and S1[0] == np.float32(1.0)  # 1 + 2^-24 rounds to 1
    assert S2[0] == 0.0  # and not 2^-24


def test_planted_sign_error_is_caught(monkeypatch):
    A = ints(401, 12, 10)
    B = ints(402, 10, 14)

    def bad_preadd_a(A11, A12, A21, A22):
        S1 = A21 + A22
        S2 = S1 - A11
        S3 = A21 - A11  # wrong sign
        S4 = A12 - S2
        return S1, S2, S3, S4

    monkeypatch.setattr(W, "preadd_a", bad_preadd_a)
    assert not np.array_equal(W.winograd(A, B, 1), classic.gemm(A, B))


def test_planted_operand_swap_is_caught(monkeypatch):
    A = ints(403, 12, 10)
    B = ints(404, 10, 14)
    good = W.product_pairs

    def bad_pairs(A11, A12, A22, B11, B21, B22, S, T):
        pairs = good(A11, A12, A22, B11, B21, B22, S, T)
        pairs[1] = (A12, B11)  # P2 should use B21
        return pairs

    monkeypatch.setattr(W, "product_pairs", bad_pairs)
    assert not np.array_equal(W.winograd(A, B, 1), classic.gemm(A, B))


def test_certificate_small_integers():
    A = ints(501, 128, 128, -1, 1)
    B = ints(502, 128, 128, -1, 1)
    cert = W.Certificate()
    W.winograd(A, B, 3, 1, cert)
    assert cert.exact_in_fp32 and cert.leaves == 343
    big = ints(503, 64, 64, -5000, 5000)
    cert2 = W.Certificate()
    W.winograd(big, big, 1, 1, cert2)
    assert not cert2.exact_in_fp32


# ---------------------------------------------------------------- structure

def test_structure_closed_forms():
    s = W.structure(19456, 19456, 19456, 3, 1024)
    assert s["depth"] == 3 and s["leaves"] == 343 and s["leaf_dims"] == (2432, 2432, 2432)
    assert s["leaf_flops"] == int(2 * 19456 ** 3 * (7 / 8) ** 3)
    # 27 n_l^2 bytes per square node at level l's child extent: 32+32+44 = 108 = 4*27
    exp = sum(7 ** l * 108 * (19456 // 2 ** (l + 1)) ** 2 for l in range(3))
    assert s["add_bytes"] == exp
    assert W.effective_depth(4096, 4096, 4096, 3, 1024) == 2
    assert W.effective_depth(19456, 16384, 12288, 4, 1024) == 3
    assert W.effective_depth(19456, 16384, 12288, 4, 768) == 4
    assert W.effective_depth(6015, 6015, 6015, 9, 3008) == 0   # paper: stop below 6016
    assert W.effective_depth(6016, 6016, 6016, 9, 3008) == 1
    # structure(M, N, K, ...) reports leaf extents as (m, k, n)
    assert W.structure(5, 7, 9, 1, 1)["leaf_dims"] == (3, 5, 4)


# ---------------------------------------------------------------- Table 1 and eqs. (3)-(4)

@pytest.mark.parametrize("m,k,n", [(8, 8, 8), (13, 9, 7), (21, 30, 17)])
def test_rmul_table1_and_two_device_split(m, k, n):
    A = ints(601, m, k)
    B = ints(602, k, n)
    ref = classic.gemm(A, B)
    for d in range(4):
        assert np.array_equal(W.rmul(A, B, d), ref)
    C = ints(603, m, n)
    acc = C.copy()
    W.rmul_add(acc, A, B, 2)
    assert np.array_equal(acc, C + ref)
    left, right = W.two_device_split(A, B)
    assert np.array_equal(np.concatenate([left, right], axis=1), ref)


# ---------------------------------------------------------------- checks

def test_rel_frob_and_freivalds_detect_missing_block():
    A = synthgen.uniform_pm1_np(701, 64, 48)
    B = synthgen.uniform_pm1_np(702, 48, 56)
    C = classic.gemm(A, B).astype(np.float32)
    x = synthgen.signs_pm1(703, 56)
    assert checks.freivalds_rel(C, A, B, x) < 1e-6
    assert checks.sampled_rows_rel(C, A, B, np.arange(64)) == pytest.approx(
        checks.rel_frob(C, classic.gemm(A, B)))
    bad = C.copy()
    bad[32:, 28:] = 0.0
    assert checks.freivalds_rel(bad, A, B, x) > 0.1
    assert checks.rel_frob(bad, classic.gemm(A, B)) > 0.1


# ---------------------------------------------------------------- MLP

def _mlp_case(seed=801, batch=17):
    flat = synthgen.uniform_pm1_np(seed, 1, mlp.N_PARAMS)[0].astype(np.float64) * 0.3
    X = synthgen.uniform_pm1_np(seed + 1, batch, mlp.D_IN).astype(np.float64)
    t = synthgen.uniform_pm1_np(seed + 2, 1, batch)[0].astype(np.float64)
    return flat, X, t


def test_mlp_backward_matches_finite_differences():
    flat, X, t = _mlp_case()
    y, cache = mlp.forward(flat, X)
    g = mlp.backward(flat, cache, y, t)
    gn = mlp.numeric_grad(flat, X, t)
    assert np.linalg.norm(g - gn) / np.linalg.norm(gn) < 1e-6


def test_mlp_forward_closed_forms():
    flat, X, _ = _mlp_case()
    p = mlp.unflatten(flat)
    # Zero output weights: the network outputs its last bias.
    p0 = dict(p)
    p0["W3"] = np.zeros_like(p["W3"])
    y, _ = mlp.forward(mlp.flatten(p0), X)
    assert np.all(y == p["b3"][0])
    # Non-negative weights and inputs: every ReLU is active and the network
    # is the affine map X W1 W2 W3 + (b1 W2 + b2) W3 + b3.
    q = {k: np.abs(v) for k, v in p.items()}
    Xp = np.abs(X)
    y, _ = mlp.forward(mlp.flatten(q), Xp)
    lin = Xp @ q["W1"] @ q["W2"] @ q["W3"] + (q["b1"] @ q["W2"] + q["b2"]) @ q["W3"] + q["b3"]
    np.testing.assert_allclose(y, lin[:, 0], rtol=1e-12)


def test_adam_first_step_is_signed_lr():
    flat, X, t = _mlp_case()
    y, cache = mlp.forward(flat, X)
    g = mlp.backward(flat, cache, y, t)
    z = np.zeros_like(flat)
    with np.errstate(invalid="ignore"):  # eps = 0: entries with zero gradient are 0/0
        new, m, v = mlp.adam_step(flat, g, z, z, 1, lr=1e-3, eps=0.0)
    nz = g != 0
    np.testing.assert_allclose((flat - new)[nz], 1e-3 * np.sign(g[nz]), rtol=1e-12)
