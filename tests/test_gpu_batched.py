"""fastmm_gemm_batched: uneven problems in one level-wise schedule, captured
into a HIP graph and replayed.  Every problem is checked against the oracle
(the FP64-accumulated classic product: relative Frobenius error <= 1e-4 on
uniform inputs, bit for bit on certified integers), and must also equal, bit
for bit, the same product computed alone by fastmm_gemm with the same plan."""
import numpy as np
import pytest

import synthgen
from oracle import checks, classic
from oracle import winograd as W
from tests.gpu_util import dev, empty_dev, host, ints, say, uniform

TOL = 1e-4

pytestmark = pytest.mark.gpu

SHAPES = [(256, 320, 192, 2), (513, 257, 129, 1), (64, 64, 64, 0), (1000, 30, 700, 3),
          (384, 512, 448, 3), (17, 9, 33, 1), (768, 768, 768, 2), (128, 1024, 256, 1)]


def _make(shapes, seed):
    As = [dev(uniform(seed + 3 * i, m, k)) for i, (m, k, n, d) in enumerate(shapes)]
    Bs = [dev(uniform(seed + 3 * i + 1, k, n)) for i, (m, k, n, d) in enumerate(shapes)]
    return As, Bs


def _singles(fastmm, shapes, As, Bs):
    outs = []
    for (m, k, n, d), A, B in zip(shapes, As, Bs):
        C = empty_dev(m, n)
        fastmm.gemm(m, n, k, A, B, C, depth=d, leaf=1)
        outs.append(host(C))
    return outs


def test_batched_equals_single_calls_and_replays(fastmm):
    import torch
    depths = [d for (_, _, _, d) in SHAPES]
    leaves = [1] * len(SHAPES)
    for call in range(3):
        say(f"batched call {call}")
        As, Bs = _make(SHAPES, 1300 + 100 * call)
        Cs = [empty_dev(m, n) for (m, k, n, d) in SHAPES]
        fastmm.gemm_batched(As, Bs, Cs, depth=depths, leaf=leaves)
        st = fastmm.get_stats()
        assert st["graph_replayed"] == (1 if call > 0 else 0)
        # eager work on the device between replays
        junk = torch.randn(1 << 20, device="cuda")
        junk.mul_(2.0).add_(1.0)
        torch.cuda.synchronize()
        refs = _singles(fastmm, SHAPES, As, Bs)
        for i, (C, ref) in enumerate(zip(Cs, refs)):
            got = host(C)
            assert np.array_equal(got, ref), f"call {call} problem {i}"
            err = checks.rel_frob(got, classic.gemm(host(As[i]), host(Bs[i])))
            assert err <= TOL, f"call {call} problem {i}: {err}"


def test_batched_certified_integers_exact(fastmm):
    # Entries in {-1, 0, 1}: the oracle's integer certificate shows every
    # intermediate of the recursion is an integer below 2^24, so every FP32
    # step is exact and each batched result must equal the exact product.
    shapes = SHAPES + [(1030, 770, 514, 3), (300, 900, 260, 2)]
    As = [dev(ints(3400 + 3 * i, m, k)) for i, (m, k, n, d) in enumerate(shapes)]
    Bs = [dev(ints(3401 + 3 * i, k, n)) for i, (m, k, n, d) in enumerate(shapes)]
    Cs = [empty_dev(m, n) for (m, k, n, d) in shapes]
    fastmm.gemm_batched(As, Bs, Cs, depth=[d for (_, _, _, d) in shapes], leaf=[1] * len(shapes))
    assert fastmm.get_stats()["depth"] == 3
    for i, (m, k, n, d) in enumerate(shapes):
        A = host(As[i]).astype(np.int64)
        B = host(Bs[i]).astype(np.int64)
        cert = W.Certificate()
        exact = W.winograd(A, B, d, 1, cert)
        assert cert.exact_in_fp32, i
        assert np.array_equal(exact, classic.gemm(A, B))
        assert np.array_equal(host(Cs[i]).astype(np.int64), exact), f"problem {i} {m}x{k}x{n} d{d}"


def test_batched_new_buffers_same_shapes(fastmm):
    # Same shapes, different tensors: the replay must read the new pointers.
    depths = [d for (_, _, _, d) in SHAPES]
    for seed in (1700, 1800):
        As, Bs = _make(SHAPES, seed)
        Cs = [empty_dev(m, n) for (m, k, n, d) in SHAPES]
        fastmm.gemm_batched(As, Bs, Cs, depth=depths, leaf=[1] * len(SHAPES))
        refs = _singles(fastmm, SHAPES, As, Bs)
        for i, (C, ref) in enumerate(zip(Cs, refs)):
            assert np.array_equal(host(C), ref)
            assert checks.rel_frob(host(C), classic.gemm(host(As[i]), host(Bs[i]))) <= TOL


def test_batched_graph_off_matches(fastmm, monkeypatch):
    depths = [d for (_, _, _, d) in SHAPES]
    As, Bs = _make(SHAPES, 1900)
    C1 = [empty_dev(m, n) for (m, k, n, d) in SHAPES]
    C2 = [empty_dev(m, n) for (m, k, n, d) in SHAPES]
    fastmm.gemm_batched(As, Bs, C1, depth=depths, leaf=[1] * len(SHAPES))
    monkeypatch.setenv("FASTMM_GRAPH", "0")
    fastmm.gemm_batched(As, Bs, C2, depth=depths, leaf=[1] * len(SHAPES))
    for a, b in zip(C1, C2):
        assert np.array_equal(host(a), host(b))


@pytest.mark.parametrize("graph", ["1", "0"])
def test_batched_persistent_matches_one_workgroup_per_tile(fastmm, monkeypatch, graph):
    # The persistent leaf launch (tiles taken from a device counter that the
    # kernel clears when it ends) gives the same bits as one workgroup per
    # tile, call after call (graph replays included).
    depths = [d for (_, _, _, d) in SHAPES]
    As, Bs = _make(SHAPES, 2100)
    monkeypatch.setenv("FASTMM_GRAPH", graph)
    monkeypatch.setenv("FASTMM_PERSISTENT", "0")
    ref = [empty_dev(m, n) for (m, k, n, d) in SHAPES]
    fastmm.gemm_batched(As, Bs, ref, depth=depths, leaf=[1] * len(SHAPES))
    monkeypatch.setenv("FASTMM_PERSISTENT", "1")
    for call in range(3):
        say(f"persistent batched call {call} graph={graph}")
        Cs = [empty_dev(m, n) for (m, k, n, d) in SHAPES]
        fastmm.gemm_batched(As, Bs, Cs, depth=depths, leaf=[1] * len(SHAPES))
        for a, b in zip(Cs, ref):
            assert np.array_equal(host(a), host(b))


def test_batched_host_operands(fastmm):
    import torch
    shapes = SHAPES[:5]
    depths = [d for (_, _, _, d) in shapes]
    As, Bs = _make(shapes, 2000)
    refs = _singles(fastmm, shapes, As, Bs)
    Ah = [a.cpu().pin_memory() for a in As]
    Bh = [b.cpu().pin_memory() for b in Bs]
    Ch = [torch.full((m, n), float("nan")).pin_memory() for (m, k, n, d) in shapes]
    fastmm.gemm_batched(Ah, Bh, Ch, depth=depths, leaf=[1] * len(shapes))
    for i, (C, ref) in enumerate(zip(Ch, refs)):
        assert np.array_equal(C.numpy(), ref)
        assert checks.rel_frob(C.numpy(), classic.gemm(host(As[i]), host(Bs[i]))) <= TOL


def test_batched_validation_is_atomic(fastmm):
    import torch
    shapes = SHAPES[:3]
    As, Bs = _make(shapes, 2100)
    Cs = [torch.full((m, n), 5.0, device="cuda") for (m, k, n, d) in shapes]
    M = [m for (m, k, n, d) in shapes]
    K = [k for (m, k, n, d) in shapes]
    N = [n for (m, k, n, d) in shapes]
    ldb = list(N)
    ldb[2] = N[2] - 1  # invalid: ldb < N for the last problem only
    rc = fastmm.gemm_batched_raw(M, N, K, [a.data_ptr() for a in As], K,
                                 [b.data_ptr() for b in Bs], ldb, [c.data_ptr() for c in Cs], N,
                                 depth=[1, 1, 1], leaf=[1, 1, 1])
    assert rc == fastmm.ERROR_INVALID_VALUE
    assert "problem 2" in fastmm.last_error()
    for C in Cs:
        assert torch.all(C == 5.0).item()


def test_batched_loguniform_shapes_planner(fastmm):
    # A scaled-down version of the 256-problem workload: shapes log-uniform
    # in [256, 2048], multiples of 64, depth and tile from the planner.
    shapes = synthgen.shapes_loguniform(3001, 24, lo=256, hi=2048)
    As = [dev(uniform(2200 + i, int(m), int(k))) for i, (m, n, k) in enumerate(shapes)]
    Bs = [dev(uniform(2300 + i, int(k), int(n))) for i, (m, n, k) in enumerate(shapes)]
    Cs = [empty_dev(int(m), int(n)) for (m, n, k) in shapes]
    fastmm.set_plan_mode(fastmm.PLAN_DEFAULT)
    fastmm.gemm_batched(As, Bs, Cs)
    for i, (m, n, k) in enumerate(shapes):
        ref = classic.gemm(host(As[i]), host(Bs[i]))
        assert checks.rel_frob(host(Cs[i]), ref) < 1e-4, i


def test_batched_exact_repeat_new_data_and_interleaved_call(fastmm):
    # A call that repeats the last one (same problems, pointers, plans)
    # replays its graph without planning or building again; the descriptors
    # still go to the device on every call, so new data in the same buffers
    # and another product run in between (which reuses that part of the
    # workspace) must not leave a stale result.
    import torch
    shapes = [(384, 320, 448, 1), (1024, 512, 768, 2), (256, 768, 640, 0), (768, 768, 768, 2)]
    As, Bs = _make(shapes, 9100)
    Cs = [empty_dev(m, n) for (m, k, n, d) in shapes]
    depth = [d for (_, _, _, d) in shapes]
    leaf = [64] * len(shapes)
    fastmm.gemm_batched(As, Bs, Cs, depth=depth, leaf=leaf)
    first = fastmm.get_stats()
    fastmm.gemm_batched(As, Bs, Cs, depth=depth, leaf=leaf)
    st = fastmm.get_stats()
    assert st["graph_replayed"] == 1
    assert (st["leaves"], st["launches"], st["depth"]) == (first["leaves"], first["launches"], first["depth"])
    for i, (m, k, n, d) in enumerate(shapes):
        As[i].copy_(dev(uniform(9200 + 2 * i, m, k)))
        Bs[i].copy_(dev(uniform(9201 + 2 * i, k, n)))
    say("exact repeat after new data and an interleaved single product")
    x, y = dev(uniform(9300, 512, 512)), dev(uniform(9301, 512, 512))
    z = empty_dev(512, 512)
    fastmm.gemm(512, 512, 512, x, y, z, depth=2, leaf=64)
    fastmm.gemm_batched(As, Bs, Cs, depth=depth, leaf=leaf)
    assert fastmm.get_stats()["graph_replayed"] == 1
    for i, (m, k, n, d) in enumerate(shapes):
        assert checks.rel_frob(host(Cs[i]), classic.gemm(host(As[i]), host(Bs[i]))) <= TOL, i
    assert checks.rel_frob(host(z), classic.gemm(host(x), host(y))) <= TOL


def test_batched_exact_repeat_honours_workspace_controls(fastmm, monkeypatch):
    # An exact repeat skips planning and building, but not the workspace
    # controls: a cap set between two identical calls must still fail the
    # second with OUT_OF_MEMORY, and a NaN-poisoned workspace must still give
    # the oracle's result.
    shapes = [(384, 320, 448, 1), (1024, 512, 768, 2), (768, 768, 768, 2)]
    As, Bs = _make(shapes, 9500)
    Cs = [empty_dev(m, n) for (m, k, n, d) in shapes]
    run = fastmm.Batch(As, Bs, Cs, depth=[d for (*_, d) in shapes], leaf=[64] * len(shapes))
    run()
    run()
    assert fastmm.get_stats()["graph_replayed"] == 1
    say("exact repeat under FASTMM_WORKSPACE_LIMIT=4096")
    monkeypatch.setenv("FASTMM_WORKSPACE_LIMIT", "4096")
    assert run(check=False) == fastmm.ERROR_OUT_OF_MEMORY
    assert "FASTMM_WORKSPACE_LIMIT" in fastmm.last_error()
    monkeypatch.delenv("FASTMM_WORKSPACE_LIMIT")
    say("exact repeat under FASTMM_POISON=1")
    monkeypatch.setenv("FASTMM_POISON", "1")
    for C in Cs:
        C.fill_(float("nan"))
    run()
    monkeypatch.delenv("FASTMM_POISON")
    for i, (m, k, n, d) in enumerate(shapes):
        assert checks.rel_frob(host(Cs[i]), classic.gemm(host(As[i]), host(Bs[i]))) <= TOL, i
    run()
    assert fastmm.get_stats()["graph_replayed"] == 1


def test_batch_object_matches_gemm_batched(fastmm):
    # fastmm.Batch builds the argument arrays once; each call must give
    # what fastmm.gemm_batched gives on the same lists, bit for bit.
    As, Bs = _make(SHAPES, 9400)
    C1 = [empty_dev(m, n) for (m, k, n, d) in SHAPES]
    C2 = [empty_dev(m, n) for (m, k, n, d) in SHAPES]
    depth = [d for (_, _, _, d) in SHAPES]
    fastmm.gemm_batched(As, Bs, C1, depth=depth, leaf=[1] * len(SHAPES))
    run = fastmm.Batch(As, Bs, C2, depth=depth, leaf=[1] * len(SHAPES))
    for _ in range(3):
        run()
        for a, b in zip(C1, C2):
            assert np.array_equal(host(a), host(b))
