"""End-to-end parity of fastmm_gemm (Winograd recursion + MFMA leaves)
against the oracle, through the C ABI.

Tolerances (relative Frobenius against the FP64-accumulated classic product):
2e-6 for depth 0 at n = 512, 1e-4 for Winograd depth <= 4.  Bit-exact where
the oracle's integer certificate shows every FP32 intermediate is an exact
integer below 2**24."""
import numpy as np
import pytest

import synthgen
from oracle import checks, classic
from oracle import winograd as W
from tests.gpu_util import dev, empty_dev, host, ints, say, uniform

pytestmark = pytest.mark.gpu

TOL_WINOGRAD = 1e-4


@pytest.mark.parametrize("n,depth,leaf", [(512, 1, 64), (512, 2, 64), (512, 3, 32), (1024, 4, 32),
                                          (768, 2, 128)])
def test_winograd_uniform_square(fastmm, n, depth, leaf):
    say(f"winograd n={n} depth={depth} leaf={leaf}")
    A = uniform(1001 + 2, n, n)
    B = uniform(2001 + 2, n, n)
    C = empty_dev(n, n)
    fastmm.gemm(n, n, n, dev(A), dev(B), C, depth=depth, leaf=leaf)
    st = fastmm.get_stats()
    assert st["depth"] == W.effective_depth(n, n, n, depth, leaf)
    err = checks.rel_frob(host(C), classic.gemm(A, B))
    say(f"  depth={st['depth']} rel_frob={err:.3e}")
    assert err <= TOL_WINOGRAD


@pytest.mark.parametrize("m,k,n,depth", [(257, 131, 383, 2), (33, 65, 17, 3), (101, 99, 103, 4),
                                         (200, 64, 130, 1), (97, 301, 45, 3), (3, 3, 3, 1)])
@pytest.mark.parametrize("tile", [0, 3])
def test_winograd_ragged_certified_exact(fastmm, m, k, n, depth, tile):
    say(f"winograd ragged {m}x{k}x{n} depth={depth} tile={tile}")
    A = ints(71 + m, m, k)
    B = ints(72 + n, k, n)
    cert = W.Certificate()
    ref = W.winograd(A.astype(np.int64), B.astype(np.int64), depth, 1, cert)
    assert cert.exact_in_fp32
    assert np.array_equal(ref, classic.gemm(A.astype(np.int64), B.astype(np.int64)))
    C = empty_dev(m, n)
    fastmm.gemm(m, n, k, dev(A), dev(B), C, depth=depth, leaf=1, tile=tile)
    assert fastmm.get_stats()["depth"] == W.effective_depth(m, k, n, depth, 1)
    assert np.array_equal(host(C).astype(np.int64), ref)


def test_winograd_all_ones_equals_k(fastmm):
    m, k, n = 640, 576, 704
    A = np.ones((m, k), np.float32)
    B = np.ones((k, n), np.float32)
    C = empty_dev(m, n)
    fastmm.gemm(m, n, k, dev(A), dev(B), C, depth=3, leaf=32)
    assert fastmm.get_stats()["depth"] == 3
    assert np.all(host(C) == k)


def test_structure_counts_match_closed_forms(fastmm, monkeypatch):
    M, N, K = 1536, 1024, 1280
    A = uniform(81, M, K)
    B = uniform(82, K, N)
    C = empty_dev(M, N)
    monkeypatch.setenv("FASTMM_TREE_ADDS", "1")  # one level per launch
    fastmm.gemm(M, N, K, dev(A), dev(B), C, depth=3, leaf=64)
    st = fastmm.get_stats()
    s = W.structure(M, N, K, 3, 64)
    assert st["depth"] == s["depth"] == 3
    assert st["leaves"] == s["leaves"] == 343
    assert (st["leaf_m"], st["leaf_k"], st["leaf_n"]) == s["leaf_dims"]
    assert st["leaf_flops"] == s["leaf_flops"]
    assert st["add_bytes"] == s["add_bytes"]
    assert st["launches"] == 3 * 3 + 1
    # Every split is exact: the three levels of each side take one pass
    # (the operand read once; of the S / T blocks, the cells that later
    # levels read as views: 4^3 + 4 * 3^2 + 7 * 4 * 3 + 49 * 4 = 380
    # leaf-sized cells), and so do the post-additions (343 products read,
    # the 64 cells of C written).
    monkeypatch.setenv("FASTMM_TREE_ADDS", "3")
    fastmm.gemm(M, N, K, dev(A), dev(B), C, depth=3, leaf=64)
    st = fastmm.get_stats()
    lm, lk, ln = s["leaf_dims"]
    assert st["add_bytes"] == 4 * (380 * lm * lk + 380 * lk * ln + (343 + 64) * lm * ln)
    assert st["launches"] == 4


def test_host_pinned_and_pageable_match_device(fastmm):
    import torch
    n, depth, leaf = 640, 2, 64
    A = uniform(91, n, n)
    B = uniform(92, n, n)
    Cd = empty_dev(n, n)
    fastmm.gemm(n, n, n, dev(A), dev(B), Cd, depth=depth, leaf=leaf)
    ref = host(Cd)
    exact = classic.gemm(A, B)
    # pinned host (pipelined path: within tolerance, see test_host_paths_match_device)
    Ap = torch.from_numpy(A).pin_memory()
    Bp = torch.from_numpy(B).pin_memory()
    Cp = torch.empty((n, n), dtype=torch.float32).pin_memory()
    fastmm.gemm(n, n, n, Ap, Bp, Cp, depth=depth, leaf=leaf)
    assert checks.rel_frob(Cp.numpy(), exact) < TOL_WINOGRAD
    assert fastmm.get_stats()["transfer_bytes"] == 4.0 * 3 * n * n
    # pageable host gives the same bits as pinned (same path)
    Ch = torch.zeros((n, n), dtype=torch.float32)
    fastmm.gemm(n, n, n, torch.from_numpy(A), torch.from_numpy(B), Ch, depth=depth, leaf=leaf)
    assert np.array_equal(Ch.numpy(), Cp.numpy())
    assert checks.rel_frob(ref, exact) < TOL_WINOGRAD


def test_host_strided_operands(fastmm):
    import torch
    m, k, n = 300, 260, 280
    Abig = uniform(93, m, k + 12)
    Bbig = uniform(94, k, n + 4)
    Cbig = torch.full((m, n + 8), -3.0)
    At = torch.from_numpy(Abig)
    Bt = torch.from_numpy(Bbig)
    fastmm.gemm(m, n, k, At.data_ptr(), Bt.data_ptr(), Cbig.data_ptr(), depth=2, leaf=32,
                lda=k + 12, ldb=n + 4, ldc=n + 8)
    got = Cbig.numpy()
    assert checks.rel_frob(got[:, :n], classic.gemm(Abig[:, :k], Bbig[:, :n])) < TOL_WINOGRAD
    assert np.all(got[:, n:] == -3.0)


def test_deterministic(fastmm):
    n = 896
    A = dev(uniform(95, n, n))
    B = dev(uniform(96, n, n))
    C1 = empty_dev(n, n)
    C2 = empty_dev(n, n)
    fastmm.gemm(n, n, n, A, B, C1, depth=3, leaf=64)
    fastmm.gemm(n, n, n, A, B, C2, depth=3, leaf=64)
    assert np.array_equal(host(C1), host(C2))


def test_poisoned_workspace(fastmm, monkeypatch):
    # Workspace filled with NaN before the call: any read of a temporary the
    # schedule did not write would put NaN into C.
    monkeypatch.setenv("FASTMM_POISON", "1")
    for (m, k, n, d) in [(512, 512, 512, 3), (333, 201, 257, 3)]:
        A = uniform(97, m, k)
        B = uniform(98, k, n)
        C = empty_dev(m, n)
        fastmm.gemm(m, n, k, dev(A), dev(B), C, depth=d, leaf=16)
        got = host(C)
        assert np.isfinite(got).all()
        assert checks.rel_frob(got, classic.gemm(A, B)) < TOL_WINOGRAD


@pytest.mark.parametrize("m,k,n,d", [(333, 201, 257, 3), (3000, 2000, 8195, 2), (4100, 1030, 8203, 3),
                                     (1500, 700, 900, 0), (2051, 4097, 9001, 0)])
def test_poisoned_workspace_host_pipeline(fastmm, monkeypatch, m, k, n, d):
    # The same with host operands: the pipelined path's device copies of A,
    # B and C, its temporaries and its padding all live in the poisoned
    # workspace, so a piece that read an operand block, an S / T band or a
    # shared inner temporary before the stream that writes it had done so
    # would leave NaN in C.
    import torch
    monkeypatch.setenv("FASTMM_POISON", "1")
    say(f"poisoned host pipeline {m}x{k}x{n} depth={d}")
    A = uniform(99 + m, m, k)
    B = uniform(100 + n, k, n)
    Cp = torch.full((m, n), float("nan")).pin_memory()
    fastmm.gemm(m, n, k, torch.from_numpy(A).pin_memory(), torch.from_numpy(B).pin_memory(), Cp,
                depth=d, leaf=1)
    got = Cp.numpy()
    assert np.isfinite(got).all()
    rows = synthgen.row_sample(101 + m, m, 8)
    assert checks.sampled_rows_rel(got, A, B, rows) <= TOL_WINOGRAD
    assert checks.freivalds_rel(got, A, B, synthgen.signs_pm1(102 + n, n)) <= TOL_WINOGRAD


def test_empty_and_k0(fastmm):
    import torch
    C = torch.full((4, 5), 9.0, device="cuda")
    A = torch.zeros((4, 1), device="cuda")
    B = torch.zeros((1, 5), device="cuda")
    fastmm.gemm(4, 5, 0, A.data_ptr(), B.data_ptr(), C.data_ptr(), depth=2, leaf=1,
                lda=1, ldb=5, ldc=5)
    assert torch.all(C == 0).item()
    C.fill_(9.0)
    fastmm.gemm(0, 5, 3, 0, B.data_ptr(), C.data_ptr(), depth=2, leaf=1, lda=3, ldb=5, ldc=5)
    assert torch.all(C == 9.0).item()


def test_invalid_arguments_leave_c_untouched(fastmm):
    import torch
    A = torch.ones((8, 8), device="cuda")
    B = torch.ones((8, 8), device="cuda")
    C = torch.full((8, 8), 5.0, device="cuda")
    a, b, c = A.data_ptr(), B.data_ptr(), C.data_ptr()
    cases = [
        (-1, 8, 8, a, 8, b, 8, c, 8, 0, 1),      # negative M
        (8, 8, 8, a, 7, b, 8, c, 8, 0, 1),       # lda < K
        (8, 8, 8, a, 8, b, 7, c, 8, 0, 1),       # ldb < N
        (8, 8, 8, a, 8, b, 8, c, 7, 0, 1),       # ldc < N
        (8, 8, 8, a, 8, b, 8, c, 8, 17, 1),      # depth > 16
        (8, 8, 8, 0, 8, b, 8, c, 8, 0, 1),       # NULL A
        (8, 8, 8, a, 8, b, 8, a, 8, 0, 1),       # C aliases A
    ]
    for args in cases:
        rc = fastmm.gemm_raw(*args)
        assert rc == fastmm.ERROR_INVALID_VALUE, args
        assert fastmm.last_error() != ""
        assert torch.all(C == 5.0).item()
    assert fastmm.gemm_raw(8, 8, 8, a, 8, b, 8, c, 8, 0, 1, 10) == fastmm.ERROR_INVALID_VALUE  # no tile 10


def test_mixed_residency_not_supported(fastmm):
    import torch
    A = torch.ones((8, 8), device="cuda")
    B = torch.ones((8, 8))
    C = torch.full((8, 8), 5.0, device="cuda")
    rc = fastmm.gemm_raw(8, 8, 8, A.data_ptr(), 8, B.data_ptr(), 8, C.data_ptr(), 8, 1, 1)
    assert rc == fastmm.ERROR_NOT_SUPPORTED
    assert torch.all(C == 5.0).item()


def test_workspace_limit_gives_out_of_memory(fastmm, monkeypatch):
    import torch
    n = 512
    A = dev(uniform(99, n, n))
    B = dev(uniform(100, n, n))
    C = torch.full((n, n), 5.0, device="cuda")
    monkeypatch.setenv("FASTMM_WORKSPACE_LIMIT", "4096")
    rc = fastmm.gemm_raw(n, n, n, A.data_ptr(), n, B.data_ptr(), n, C.data_ptr(), n, 2, 64)
    assert rc == fastmm.ERROR_OUT_OF_MEMORY
    assert "FASTMM_WORKSPACE_LIMIT" in fastmm.last_error()
    monkeypatch.delenv("FASTMM_WORKSPACE_LIMIT")
    fastmm.gemm(n, n, n, A, B, C, depth=2, leaf=64)
    assert torch.isfinite(C).all().item()


@pytest.mark.parametrize("n,depth,leaf", [(4096, 2, 1024), (4096, 3, 512), (8192, 3, 1024)])
def test_config2_sampled_rows_and_freivalds(fastmm, n, depth, leaf):
    say(f"config n={n} depth={depth} leaf={leaf}")
    A = uniform(1001 + 2, n, n)
    B = uniform(2001 + 2, n, n)
    C = empty_dev(n, n)
    fastmm.gemm(n, n, n, dev(A), dev(B), C, depth=depth, leaf=leaf)
    got = host(C)
    rows = synthgen.row_sample(7002, n, 48)
    e_rows = checks.sampled_rows_rel(got, A, B, rows)
    e_fv = checks.freivalds_rel(got, A, B, synthgen.signs_pm1(7003, n))
    say(f"  depth={fastmm.get_stats()['depth']} rows={e_rows:.3e} freivalds={e_fv:.3e}")
    assert e_rows <= TOL_WINOGRAD and e_fv <= TOL_WINOGRAD


@pytest.mark.parametrize("m,k,n,depth", [(640, 640, 640, 2), (333, 201, 257, 3), (300, 260, 280, 0),
                                         (97, 301, 45, 1), (2, 3, 2, 1), (1024, 512, 768, 3),
                                         (700, 300, 500, 0), (1500, 700, 900, 2)])
@pytest.mark.parametrize("pipeline", ["1", "0"])
def test_host_paths_match_device(fastmm, monkeypatch, m, k, n, depth, pipeline):
    # Host operands go through the staged path: pipelined (quadrant row bands
    # in, top level product by product, result blocks out) or copy-all-first.
    # Copy-first and every plain (depth 0) product equal the device-resident
    # result bit for bit; the pipelined Winograd path splits the inner
    # recursion by row bands (another rounding order), so it is held to the
    # oracle tolerance -- and to exactness on certified integers below.
    import torch
    say(f"host path {m}x{k}x{n} depth={depth} pipeline={pipeline}")
    monkeypatch.setenv("FASTMM_PIPELINE", pipeline)
    A = uniform(111 + m, m, k)
    B = uniform(112 + n, k, n)
    Cd = empty_dev(m, n)
    fastmm.gemm(m, n, k, dev(A), dev(B), Cd, depth=depth, leaf=1)
    ref = host(Cd)
    Ap = torch.from_numpy(A).pin_memory()
    Bp = torch.from_numpy(B).pin_memory()
    Cp = torch.full((m, n), float("nan")).pin_memory()
    fastmm.gemm(m, n, k, Ap, Bp, Cp, depth=depth, leaf=1)
    st = fastmm.get_stats()
    assert st["depth"] == W.effective_depth(m, k, n, depth, 1)
    exact = classic.gemm(A, B)
    if pipeline == "0" or st["depth"] == 0:
        assert np.array_equal(Cp.numpy(), ref)
    else:
        assert np.isfinite(Cp.numpy()).all()
        assert checks.rel_frob(Cp.numpy(), exact) < TOL_WINOGRAD
    assert checks.rel_frob(ref, exact) < TOL_WINOGRAD


@pytest.mark.parametrize("m,k,n,depth", [(333, 201, 257, 3), (97, 301, 45, 1), (1024, 512, 768, 3),
                                         (130, 66, 258, 2)])
def test_host_pipeline_certified_exact(fastmm, m, k, n, depth):
    import torch
    A = ints(121 + m, m, k)
    B = ints(122 + n, k, n)
    cert = W.Certificate()
    ref = W.winograd(A.astype(np.int64), B.astype(np.int64), depth, 1, cert)
    assert cert.exact_in_fp32
    Cp = torch.full((m, n), float("nan")).pin_memory()
    fastmm.gemm(m, n, k, torch.from_numpy(A).pin_memory(), torch.from_numpy(B).pin_memory(), Cp,
                depth=depth, leaf=1)
    assert np.array_equal(Cp.numpy().astype(np.int64), ref)


def test_depth_first_fallback_bitwise(fastmm, monkeypatch):
    # A workspace cap below the level-wise need: the scheduler runs the top
    # levels depth first (same tree, same arithmetic), so the result must be
    # bit for bit the level-wise one; below the depth-first minimum it must
    # report OUT_OF_MEMORY with C untouched.
    import torch
    n, depth, leaf = 1024, 3, 32
    A = dev(uniform(131, n, n))
    B = dev(uniform(132, n, n))
    C0 = empty_dev(n, n)
    monkeypatch.delenv("FASTMM_WORKSPACE_LIMIT", raising=False)
    fastmm.gemm(n, n, n, A, B, C0, depth=depth, leaf=leaf)
    ref = host(C0)
    bfs_launches = fastmm.get_stats()["launches"]
    ok = 0
    for limit in [80_000_000, 50_000_000, 35_000_000, 28_000_000, 22_000_000, 18_000_000,
                  14_000_000, 10_000_000]:
        monkeypatch.setenv("FASTMM_WORKSPACE_LIMIT", str(limit))
        C = torch.full((n, n), 7.0, device="cuda")
        rc = fastmm.gemm_raw(n, n, n, A.data_ptr(), n, B.data_ptr(), n, C.data_ptr(), n, depth, leaf)
        if rc == fastmm.ERROR_OUT_OF_MEMORY:
            assert torch.all(C == 7.0).item()
            break
        assert rc == fastmm.SUCCESS, fastmm.last_error()
        st = fastmm.get_stats()
        say(f"  limit {limit}: launches {st['launches']} (level-wise {bfs_launches})")
        assert st["depth"] == depth and st["leaves"] == 343
        assert np.array_equal(host(C), ref)
        if st["launches"] > bfs_launches:
            ok += 1
    assert ok >= 2


@pytest.mark.parametrize("m,k,n,depth", [(301, 257, 203, 0), (513, 259, 387, 1), (700, 645, 1021, 2),
                                         (1030, 1031, 1029, 3)])
def test_misaligned_device_operands_staged(fastmm, m, k, n, depth):
    # Device operands whose rows are not 16-byte aligned (base offset by one
    # float, odd leading dimensions, K and N not multiples of 4) are staged
    # into padded buffers: exact on certified integers, A and B untouched,
    # nothing written outside C.
    import torch
    A = ints(141 + m, m, k)
    B = ints(142 + n, k, n)
    cert = W.Certificate()
    ref = W.winograd(A.astype(np.int64), B.astype(np.int64), depth, 1, cert)
    assert cert.exact_in_fp32
    Abig = torch.zeros(m * (k + 3) + 1, device="cuda")
    Bbig = torch.zeros(k * (n + 5) + 1, device="cuda")
    Abig[1:].view(m, k + 3)[:, :k] = dev(A)
    Bbig[1:].view(k, n + 5)[:, :n] = dev(B)
    A0, B0 = Abig.clone(), Bbig.clone()
    C = torch.full((m, n + 2), float("nan"), device="cuda")
    say(f"misaligned device operands {m}x{k}x{n} depth={depth}")
    fastmm.gemm(m, n, k, Abig.data_ptr() + 4, Bbig.data_ptr() + 4, C.data_ptr(), depth=depth,
                leaf=1, lda=k + 3, ldb=n + 5, ldc=n + 2)
    got = host(C)
    assert np.array_equal(got[:, :n].astype(np.int64), ref)
    assert np.all(np.isnan(got[:, n:]))
    assert torch.equal(Abig, A0) and torch.equal(Bbig, B0)



_FRESH_DEPTH_FIRST = r"""
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
import synthgen
from paper_1205_2927_amd import fastmm
fastmm.load()
n, depth, leaf = 1024, 3, 32
A = torch.from_numpy(synthgen.uniform_pm1(133, n, n)).to("cuda")
B = torch.from_numpy(synthgen.uniform_pm1(134, n, n)).to("cuda")
C = torch.full((n, n), float("nan"), device="cuda")
print("fresh process: first call depth-first", flush=True)
fastmm.gemm(n, n, n, A, B, C, depth=depth, leaf=leaf)
st = fastmm.get_stats()
np.save(sys.argv[2], C.cpu().numpy())
print(f"launches {st['launches']} leaves {st['leaves']} depth {st['depth']}", flush=True)
"""


def test_depth_first_fallback_first_call_in_fresh_process(fastmm, tmp_path):
    # The first call of a process runs depth first at the top and level-wise
    # below it: the children's descriptor blocks (49 leaves each) outgrow the
    # 4 KB pinned block the top level took first, so the pinned buffer is
    # reallocated while the top level still has its post-addition node to
    # upload.  The result must match the oracle and equal the level-wise one.
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = str(tmp_path / "c.npy")
    env = dict(os.environ, FASTMM_WORKSPACE_LIMIT="35000000")
    say("fresh subprocess: depth-first fallback as its first call")
    r = subprocess.run([sys.executable, "-c", _FRESH_DEPTH_FIRST, root, out], env=env,
                       capture_output=True, text=True, timeout=300)
    say(r.stdout + r.stderr[-2000:])
    assert r.returncode == 0
    launches = int(r.stdout.split("launches ")[1].split()[0])
    n = 1024
    A = uniform(133, n, n)
    B = uniform(134, n, n)
    got = np.load(out)
    C0 = empty_dev(n, n)
    fastmm.gemm(n, n, n, dev(A), dev(B), C0, depth=3, leaf=32)
    assert launches > fastmm.get_stats()["launches"]  # it did run depth first
    assert np.array_equal(got, host(C0))
    assert checks.rel_frob(got, classic.gemm(A, B)) <= TOL_WINOGRAD


@pytest.mark.parametrize("M,K,N,depth", [(3000, 2000, 8195, 2), (4100, 1030, 8203, 3), (2051, 4097, 9001, 1),
                                         (8195, 1030, 8203, 2), (9001, 515, 8199, 1)])
def test_host_pipeline_column_bands_odd_exact(fastmm, M, K, N, depth):
    # Host operands wide enough for the pipelined path's column bands of B
    # (B's quadrants at least 4096 wide), with odd extents: clipped right
    # and bottom quadrants, padded device copies.  Entries in {-1, 0, 1} keep
    # every FP32 step exact (|intermediates| far below 2^24 for K <= 4097
    # and depth <= 3), so sampled rows and Freivalds' check must be exact.
    import torch
    say(f"pipelined column bands {M}x{K}x{N} depth={depth}")
    A = ints(151 + M, M, K)
    B = ints(152 + N, K, N)
    Cp = torch.full((M, N), float("nan")).pin_memory()
    fastmm.gemm(M, N, K, torch.from_numpy(A).pin_memory(), torch.from_numpy(B).pin_memory(), Cp,
                depth=depth, leaf=1)
    assert fastmm.get_stats()["depth"] == depth
    C = Cp.numpy()
    assert np.isfinite(C).all()
    rows = synthgen.row_sample(153 + M, M, 16)
    assert np.array_equal(C[rows].astype(np.float64), classic.gemm_rows(A, B, rows))
    x = synthgen.signs_pm1(154 + N, N)
    assert np.array_equal(classic.gemv(C, x), classic.gemv(A, classic.gemv(B, x)))


@pytest.mark.parametrize("M,K,N,depth", [(333, 201, 257, 3), (1024, 512, 768, 3), (3000, 2000, 8195, 2),
                                         (4100, 1030, 8203, 3), (2051, 4097, 9001, 1)])
def test_host_pipeline_two_streams_bitwise(fastmm, monkeypatch, M, K, N, depth):
    # The pipelined path's pieces alternate between two compute streams by
    # default; every piece computes the same values in the same order either
    # way, so the result equals the one-stream schedule's bit for bit, on
    # every one of repeated calls (a missing cross-stream wait would show as
    # a result that changes from call to call), and the oracle's.
    import torch
    say(f"two compute streams {M}x{K}x{N} depth={depth}")
    A = uniform(161 + M, M, K)
    B = uniform(162 + N, K, N)
    Ap = torch.from_numpy(A).pin_memory()
    Bp = torch.from_numpy(B).pin_memory()
    monkeypatch.setenv("FASTMM_PIPE_STREAMS", "1")
    C1 = torch.full((M, N), float("nan")).pin_memory()
    fastmm.gemm(M, N, K, Ap, Bp, C1, depth=depth, leaf=1)
    one = fastmm.get_stats()
    monkeypatch.delenv("FASTMM_PIPE_STREAMS")
    for rep in range(3):
        C2 = torch.full((M, N), float("nan")).pin_memory()
        fastmm.gemm(M, N, K, Ap, Bp, C2, depth=depth, leaf=1)
        st = fastmm.get_stats()
        assert st["leaf_launches"] == one["leaf_launches"] and st["leaves"] == one["leaves"]
        assert np.array_equal(C2.numpy(), C1.numpy()), f"call {rep}"
    rows = synthgen.row_sample(163 + M, M, 8)
    assert checks.sampled_rows_rel(C1.numpy(), A, B, rows) <= TOL_WINOGRAD
    assert checks.freivalds_rel(C1.numpy(), A, B, synthgen.signs_pm1(164 + N, N)) <= TOL_WINOGRAD


@pytest.mark.parametrize("rows,cols", [(2, 2), (3, 2), (4, 2), (5, 2), (6, 2), (8, 2), (4, 3), (4, 4)])
def test_host_pipeline_band_layouts_exact(fastmm, monkeypatch, rows, cols):
    # Every band layout with an input order of its own (the top quadrants'
    # rows in `rows` bands, B's columns in `cols` bands): pieces, shared
    # inner temporaries, banded S / T passes and result blocks must still
    # give the exact product on certified integers.
    import torch
    M, K, N, depth = 4096, 1030, 8200, 2
    monkeypatch.setenv("FASTMM_PIPE_ROWBANDS", str(rows))
    monkeypatch.setenv("FASTMM_PIPE_COLBANDS", str(cols))
    say(f"band layout {rows}x{cols}: {M}x{K}x{N} depth={depth}")
    A = ints(171 + rows, M, K)
    B = ints(172 + cols, K, N)
    Cp = torch.full((M, N), float("nan")).pin_memory()
    fastmm.gemm(M, N, K, torch.from_numpy(A).pin_memory(), torch.from_numpy(B).pin_memory(), Cp,
                depth=depth, leaf=1)
    st = fastmm.get_stats()
    assert st["depth"] == depth and st["leaf_launches"] == 7 * rows * cols
    C = Cp.numpy()
    rows_s = synthgen.row_sample(173, M, 16)
    assert np.array_equal(C[rows_s].astype(np.float64), classic.gemm_rows(A, B, rows_s))
    x = synthgen.signs_pm1(174, N)
    assert np.array_equal(classic.gemv(C, x), classic.gemv(A, classic.gemv(B, x)))


@pytest.mark.parametrize("M,K,N,parts,pieces", [(10241, 515, 10243, None, 25), (10240, 512, 10752, None, 25),
                                                (1000, 300, 1003, "1", None), (1000, 300, 1003, "3", None),
                                                (1000, 300, 1003, "5", None), (1000, 300, 1003, "8", None),
                                                (9001, 257, 10240, None, 16), (4000, 300, 4100, None, 4),
                                                (6000, 300, 5000, None, 9), (7169, 130, 3000, None, 16)])
def test_host_plain_bands_bitwise(fastmm, monkeypatch, M, K, N, parts, pieces):
    # The plain product from host memory streams A's rows and B's columns in
    # bands (halves, thirds, quarters or fifths by size, or
    # FASTMM_PIPE_PLAINBANDS parts) and computes each block C[r, c] as a
    # piece: every element is still the device-resident product's, bit for
    # bit, whatever the bands.
    import torch
    if parts is None:
        monkeypatch.delenv("FASTMM_PIPE_PLAINBANDS", raising=False)
    else:
        monkeypatch.setenv("FASTMM_PIPE_PLAINBANDS", parts)
    say(f"plain bands {M}x{K}x{N} parts={parts}")
    A = uniform(181 + M, M, K)
    B = uniform(182 + N, K, N)
    Cd = empty_dev(M, N)
    fastmm.gemm(M, N, K, dev(A), dev(B), Cd, depth=0, leaf=1)
    Cp = torch.full((M, N), float("nan")).pin_memory()
    fastmm.gemm(M, N, K, torch.from_numpy(A).pin_memory(), torch.from_numpy(B).pin_memory(), Cp,
                depth=0, leaf=1)
    st = fastmm.get_stats()
    assert st["depth"] == 0
    if pieces is not None:  # one leaf launch per piece
        assert st["leaf_launches"] == pieces
    assert np.array_equal(Cp.numpy(), host(Cd))
    rows = synthgen.row_sample(183, M, 8)
    assert checks.sampled_rows_rel(Cp.numpy(), A, B, rows) <= 2e-6
