"""The planner's fixed rule and the workspace it reports, on the host (the
DEFAULT mode needs no device): depth from the stop rule with leaf cutoff
1280, 64x64 tiles for launches of fewer than 512 tiles of 128x128, and the
level-wise schedule's temporaries against their closed form."""
import pytest

from paper_1205_2927_amd import fastmm


@pytest.fixture(scope="module", autouse=True)
def lib():
    fastmm.load()


@pytest.mark.parametrize("n,depth,tile", [(19456, 3, 0), (16384, 3, 0), (10240, 3, 0), (8192, 2, 0),
                                          (5632, 2, 0), (4096, 1, 0), (3072, 1, 0), (2560, 1, 0),
                                          (2048, 0, 3), (512, 0, 3)])
def test_default_rule_on_host(n, depth, tile):
    p = fastmm.plan(n, n, n, fastmm.PLAN_DEFAULT)
    assert (p.depth, p.leaf, p.tile, p.source) == (depth, 1280, tile, fastmm.PLAN_DEFAULT)


def _closed_form_temp_bytes(n, d):
    # Level l (0..d-1) of a square product whose halves stay exact: 7^l nodes,
    # each with 4 S and 4 T blocks of (n / 2^(l+1))^2; products P of level l
    # (1..d): 7^l blocks of (n / 2^l)^2.  FP32.
    floats = 0
    for l in range(d):
        h = n >> (l + 1)
        floats += 2 * 7 ** l * 4 * h * h
    for l in range(1, d + 1):
        h = n >> l
        floats += 7 ** l * h * h
    return 4 * floats


@pytest.mark.parametrize("n", [19456, 16384, 8192, 4096])
def test_plan_workspace_matches_closed_form(n):
    p = fastmm.plan(n, n, n, fastmm.PLAN_DEFAULT)
    assert p.workspace_bytes == _closed_form_temp_bytes(n, p.depth)


def test_plan_workspace_grows_with_padding():
    # K and N rounded up to 4 (as staged operands are): never below the
    # aligned size's own temporaries
    a = fastmm.plan(6016, 6016, 6016, fastmm.PLAN_DEFAULT)
    b = fastmm.plan(6015, 6015, 6015, fastmm.PLAN_DEFAULT)
    assert a.depth == b.depth == 2
    assert a.workspace_bytes == _closed_form_temp_bytes(6016, 2)
    assert b.workspace_bytes >= _closed_form_temp_bytes(6016, 2) * 6015 // 6016


def _leaf_first_extents(m, d):
    # The engine's split rule for a d-level recursion: the leaf extent is
    # ceil(m / 2^d), rounded up to a multiple of 4 when it is 64 or more and
    # to an even number when it is 32 or more (d >= 2), so that every level's
    # extent of 64 or more is a multiple of 4; level l >= 1 is 2^(d-l) leaves.
    leaf = -(-m // 2 ** d)
    g = 4 if leaf >= 64 else (2 if d >= 2 and leaf >= 32 else 1)
    leaf = -(-leaf // g) * g
    return [m] + [leaf << (d - l) for l in range(1, d + 1)]


def _leaf_first_temp_bytes(M, N, K, d):
    # S and T blocks of levels 0..d-1 and products of levels 1..d, each
    # level's array 256-byte aligned (64 floats).
    al = lambda f: -(-f // 64) * 64
    m, k, n = (_leaf_first_extents(x, d) for x in (M, K, N))
    floats = 0
    for l in range(d):
        floats += al(7 ** l * 4 * m[l + 1] * k[l + 1]) + al(7 ** l * 4 * k[l + 1] * n[l + 1])
    for l in range(1, d + 1):
        floats += al(7 ** l * m[l] * n[l])
    return 4 * floats


@pytest.mark.parametrize("M,N,K", [(10004, 10004, 10004), (14004, 14004, 14004), (6015, 6015, 6015),
                                   (12031, 9000, 7777), (19456, 19456, 19456)])
def test_plan_workspace_follows_leaf_first_split(M, N, K):
    # Extents that do not halve exactly: every level below the top is exactly
    # twice the next (K and N first rounded up to 4, as staged operands are).
    p = fastmm.plan(M, N, K, fastmm.PLAN_DEFAULT)
    assert p.depth >= 1
    K4, N4 = -(-K // 4) * 4, -(-N // 4) * 4
    assert p.workspace_bytes == _leaf_first_temp_bytes(M, N4, K4, p.depth)


def test_leaf_first_extents_keep_the_bottom_quadrant():
    # the top split leaves a non-empty bottom quadrant, covers ceil(m/2), and
    # every extent of 64 or more is a multiple of 4
    for m in range(2, 5000, 7):
        for d in range(1, 6):
            if (m >> (d - 1)) < 2:
                continue
            e = _leaf_first_extents(m, d)
            assert (m + 1) // 2 <= e[1] < m
            assert all(x % 4 == 0 for x in e[1:] if x >= 64)
            assert all(e[l] == 2 * e[l + 1] for l in range(1, d))
