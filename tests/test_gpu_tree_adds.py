"""Multi-level additions: where every split of two or three consecutive
levels is exact, their pre-additions (and post-additions) run as one pass
that follows each element position through all of those levels.  The
chains are the single-level ones, so the result must equal, bit for bit,
the one-level-per-launch schedule (FASTMM_TREE_ADDS=1), on the level-wise
path, the batched graph, the pipelined host path and the split-precision
forms; and it must still meet the oracle's tolerance."""
import numpy as np
import pytest

from oracle import checks, classic
from tests.gpu_util import dev, empty_dev, host, say, uniform

pytestmark = pytest.mark.gpu


def _run(fastmm, monkeypatch, levels, m, k, n, A, B, depth, leaf, tile=None):
    monkeypatch.setenv("FASTMM_TREE_ADDS", str(levels))
    C = empty_dev(m, n)
    fastmm.gemm(m, n, k, A, B, C, depth=depth, leaf=leaf, tile=tile)
    return host(C), fastmm.get_stats()


# (m, k, n, depth, leaf, launches with one level per launch, launches grouped)
CASES = [
    (512, 512, 512, 2, 32, 7, 4),        # one group of 2 levels per side and for the post-additions
    (512, 512, 512, 3, 32, 10, 4),       # one group of 3
    (1536, 1024, 1280, 3, 64, 10, 4),    # rectangular
    (1024, 1024, 1024, 4, 32, 13, 7),    # top level alone, then a group of 3
    (768, 640, 896, 2, 32, 7, 4),
    (2048, 256, 1024, 3, 16, 10, 4),
]


@pytest.mark.parametrize("m,k,n,depth,leaf,n_level,n_tree", CASES)
def test_tree_adds_bitwise_equal_level_wise(fastmm, monkeypatch, m, k, n, depth, leaf, n_level, n_tree):
    say(f"tree adds {m}x{k}x{n} depth {depth}")
    A = uniform(5101 + m, m, k)
    B = uniform(5102 + n, k, n)
    Ad, Bd = dev(A), dev(B)
    ref, st1 = _run(fastmm, monkeypatch, 1, m, k, n, Ad, Bd, depth, leaf)
    got, st3 = _run(fastmm, monkeypatch, 3, m, k, n, Ad, Bd, depth, leaf)
    say(f"  launches {st1['launches']} -> {st3['launches']}, add bytes "
        f"{st1['add_bytes'] / 1e6:.1f} -> {st3['add_bytes'] / 1e6:.1f} MB")
    assert st1["depth"] == st3["depth"] == depth
    assert st1["launches"] == n_level and st3["launches"] == n_tree
    assert st3["add_bytes"] < st1["add_bytes"]
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert checks.rel_frob(got, classic.gemm(A, B)) <= 1e-4


def test_tree_adds_two_level_groups(fastmm, monkeypatch):
    # FASTMM_TREE_ADDS=2 at depth 3: a lone top level, then a group of two
    m = k = n = 512
    A, B = uniform(5201, m, k), uniform(5202, k, n)
    Ad, Bd = dev(A), dev(B)
    ref, _ = _run(fastmm, monkeypatch, 1, m, k, n, Ad, Bd, 3, 32)
    got, st = _run(fastmm, monkeypatch, 2, m, k, n, Ad, Bd, 3, 32)
    assert st["launches"] == 7
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("m,k,n,depth", [(520, 512, 512, 2), (512, 516, 512, 3), (512, 512, 508, 3),
                                         (1000, 1000, 1000, 3), (1001, 999, 1003, 2), (6015, 517, 1234, 3)])
def test_tree_adds_clipped_top(fastmm, monkeypatch, m, k, n, depth):
    # Extents that do not halve exactly: the split rule places the leaf
    # first, so only the top node's quadrants are clipped; the grouped
    # pre-addition pass reads the missing rows and columns as zero (one
    # launch per side).  A clipped C keeps the root's post-additions in the
    # single-level kernel, the levels below it grouped: 4 or 5 launches.
    A, B = uniform(5301 + m, m, k), uniform(5302 + n, k, n)
    Ad, Bd = dev(A), dev(B)
    ref, st1 = _run(fastmm, monkeypatch, 1, m, k, n, Ad, Bd, depth, 16)
    got, st3 = _run(fastmm, monkeypatch, 3, m, k, n, Ad, Bd, depth, 16)
    say(f"  {m}x{k}x{n} d{depth}: launches {st1['launches']} -> {st3['launches']}")
    assert st1["depth"] == st3["depth"] == depth
    assert st1["launches"] == 3 * depth + 1 and st3["launches"] in (4, 5)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    assert checks.rel_frob(got, classic.gemm(A, B)) <= 1e-4


@pytest.mark.parametrize("tile", [8, 9])
def test_tree_adds_split_forms(fastmm, monkeypatch, tile):
    # depth 3 with split-precision leaves: the last level's pre-additions
    # stay fused with the pack pass, the two above form one group.
    m = k = n = 1024
    A, B = uniform(5401, m, k), uniform(5402, k, n)
    Ad, Bd = dev(A), dev(B)
    ref, st1 = _run(fastmm, monkeypatch, 1, m, k, n, Ad, Bd, 3, 64, tile)
    got, st3 = _run(fastmm, monkeypatch, 3, m, k, n, Ad, Bd, 3, 64, tile)
    say(f"  tile {tile}: launches {st1['launches']} -> {st3['launches']}")
    assert st3["launches"] < st1["launches"]
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_tree_adds_batched_graph(fastmm, monkeypatch):
    import torch
    shapes = [(384, 512, 448, 3), (256, 256, 256, 2), (320, 192, 128, 1), (513, 257, 129, 2),
              (1024, 512, 768, 3)]
    As = [dev(uniform(5500 + 2 * i, m, k)) for i, (m, k, n, d) in enumerate(shapes)]
    Bs = [dev(uniform(5501 + 2 * i, k, n)) for i, (m, k, n, d) in enumerate(shapes)]
    depths = [d for (_, _, _, d) in shapes]
    out = {}
    for levels in (1, 3):
        monkeypatch.setenv("FASTMM_TREE_ADDS", str(levels))
        for call in range(2):
            Cs = [empty_dev(m, n) for (m, k, n, d) in shapes]
            fastmm.gemm_batched(As, Bs, Cs, depth=depths, leaf=[1] * len(shapes))
            assert fastmm.get_stats()["graph_replayed"] == call
            junk = torch.randn(1 << 18, device="cuda")
            junk.mul_(2.0)
            torch.cuda.synchronize()
            res = [host(C) for C in Cs]
            if call == 0:
                out[levels] = res
            else:
                for a, b in zip(res, out[levels]):
                    assert np.array_equal(a, b)
    for i, (a, b) in enumerate(zip(out[1], out[3])):
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"problem {i}"


def test_tree_adds_pinned_host(fastmm, monkeypatch):
    import torch
    n, depth = 1024, 3
    A, B = uniform(5601, n, n), uniform(5602, n, n)
    Ap = torch.from_numpy(A).pin_memory()
    Bp = torch.from_numpy(B).pin_memory()
    res = {}
    for levels in (1, 3):
        monkeypatch.setenv("FASTMM_TREE_ADDS", str(levels))
        Cp = torch.empty((n, n), dtype=torch.float32).pin_memory()
        fastmm.gemm(n, n, n, Ap, Bp, Cp, depth=depth, leaf=64)
        res[levels] = Cp.numpy().copy()
    assert np.array_equal(res[1].view(np.uint32), res[3].view(np.uint32))
    assert checks.rel_frob(res[3], classic.gemm(A, B)) <= 1e-4


@pytest.mark.parametrize("m,k,n,depth,tile,levels", [(1024, 1024, 1024, 4, None, 3), (1536, 1024, 1280, 3, None, 2),
                                                     (1024, 1024, 1024, 3, 8, 3), (1024, 1024, 1024, 3, 9, 3)])
def test_tree_adds_poisoned_workspace(fastmm, monkeypatch, m, k, n, depth, tile, levels):
    # The workspace is filled with NaN before the call: S / T cells that the
    # grouped pass does not write must never be read.
    monkeypatch.setenv("FASTMM_POISON", "1")
    A, B = uniform(5701 + m, m, k), uniform(5702 + n, k, n)
    Ad, Bd = dev(A), dev(B)
    got, st = _run(fastmm, monkeypatch, levels, m, k, n, Ad, Bd, depth, 32, tile)
    assert st["depth"] == depth
    assert np.isfinite(got).all()
    ref, _ = _run(fastmm, monkeypatch, 1, m, k, n, Ad, Bd, depth, 32, tile)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_tree_adds_batched_mixed_widths_and_clipping(fastmm, monkeypatch):
    # One batch whose level-0 launches mix 16-byte and 4-byte cells (C with a
    # leading dimension that is not a multiple of 4 takes the narrow form),
    # clipped and unclipped top operands: every problem must equal, bit for
    # bit, the same product computed alone one level per launch.
    shapes = [(1024, 1024, 1024, 2), (1001, 999, 1003, 2), (768, 640, 896, 2), (1000, 1000, 1000, 3),
              (1024, 512, 768, 3)]
    As = [dev(uniform(5800 + 2 * i, m, k)) for i, (m, k, n, d) in enumerate(shapes)]
    Bs = [dev(uniform(5801 + 2 * i, k, n)) for i, (m, k, n, d) in enumerate(shapes)]
    Cs = [empty_dev(m, n) for (m, k, n, d) in shapes]
    monkeypatch.setenv("FASTMM_TREE_ADDS", "3")
    fastmm.gemm_batched(As, Bs, Cs, depth=[d for (_, _, _, d) in shapes], leaf=[1] * len(shapes))
    got = [host(C) for C in Cs]
    monkeypatch.setenv("FASTMM_TREE_ADDS", "1")
    for i, ((m, k, n, d), A, B) in enumerate(zip(shapes, As, Bs)):
        C = empty_dev(m, n)
        fastmm.gemm(m, n, k, A, B, C, depth=d, leaf=1)
        assert np.array_equal(got[i].view(np.uint32), host(C).view(np.uint32)), f"problem {i}"


def test_tree_adds_random_shapes(fastmm, monkeypatch):
    # Seeded random extents in [1, 700] and depths 1-4 (as deep as the stop
    # rule allows with leaf 1): clipped tops, narrow and wide cells, staged
    # operands.  Integer operands in [-2, 2]: the oracle's certificate shows
    # every intermediate of these seeds to be an exact FP32 integer (far
    # below 2^24), so both schedules must equal the int64 product.
    import synthgen
    ext = synthgen.int_range(5901, 40, 3, 1, 700).astype(np.int64)
    dep = synthgen.int_range(5902, 40, 1, 1, 4)[:, 0].astype(np.int64)
    for i in range(40):
        m, k, n = (int(x) for x in ext[i])
        depth = int(dep[i])
        A = synthgen.int_range(5903 + i, m, k, -2, 2)
        B = synthgen.int_range(6003 + i, k, n, -2, 2)
        Ad, Bd = dev(A), dev(B)
        ref, st1 = _run(fastmm, monkeypatch, 1, m, k, n, Ad, Bd, depth, 1)
        got, st3 = _run(fastmm, monkeypatch, 3, m, k, n, Ad, Bd, depth, 1)
        say(f"  {m}x{k}x{n} depth {st3['depth']}: launches {st1['launches']} -> {st3['launches']}")
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (m, k, n, depth)
        assert np.array_equal(got.astype(np.int64), classic.gemm(A.astype(np.int64), B.astype(np.int64)))
