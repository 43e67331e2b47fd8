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
