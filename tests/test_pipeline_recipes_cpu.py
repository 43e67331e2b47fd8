"""Host logic of the pipelined host-operand path: the input orders of its
band layouts (the recipe table in csrc/pipeline.cpp).  Every layout's order
must bring each band block of the eight top-level quadrants (A: four
quadrants x row bands, B: four quadrants x column bands) to the device
exactly once, or a piece would read a block that was never copied."""
import os
import re

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_1205_2927_amd", "csrc", "pipeline.cpp")


def _recipes():
    with open(CSRC) as f:
        src = f.read()
    body = src[src.index("const std::vector<Recipe>& recipes()"):src.index("const Recipe* find_recipe")]
    out = {}
    for m in re.finditer(r"\{(\d+),\s*(\d+),\s*\{((?:\s*\{\d+,\s*\d+,\s*\d+\},?)+)\s*\}\}", body):
        nr, nc = int(m.group(1)), int(m.group(2))
        items = [tuple(int(x) for x in t) for t in re.findall(r"\{(\d+),\s*(\d+),\s*(\d+)\}", m.group(3))]
        assert (nr, nc) not in out, (nr, nc)
        out[(nr, nc)] = items
    return out


def test_every_layout_has_an_order():
    got = set(_recipes())
    assert got == {(2, 2), (2, 1), (4, 2), (6, 2), (8, 2), (3, 2), (5, 2), (4, 3), (4, 4)}


def test_each_order_copies_every_block_once():
    for (nr, nc), items in _recipes().items():
        want = {(0, q, b) for q in range(4) for b in range(nr)} | {(1, q, c) for q in range(4) for c in range(nc)}
        assert len(items) == len(want), (nr, nc)
        assert set(items) == want, (nr, nc)
        assert nr <= 8 and nc <= 8  # kMaxBands


def test_layouts_start_with_a_complete_piece_early():
    # The orders were searched so that the first product piece can start
    # after a few blocks: within the first three blocks there is a row band
    # of some A quadrant and a column band of some B quadrant.
    for (nr, nc), items in _recipes().items():
        first = items[:3]
        assert any(m == 0 for m, _, _ in first) and any(m == 1 for m, _, _ in first), (nr, nc)
