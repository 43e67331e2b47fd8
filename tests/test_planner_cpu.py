"""Planner host logic that needs no GPU: the timing-database file format."""
import pytest


def test_db_roundtrip_and_malformed(tmp_path):
    from paper_1205_2927_amd import fastmm
    fastmm.load()
    good = tmp_path / "db.json"
    good.write_text('{"device": "gfx950", "records": [\n'
                    '  {"M": 256, "N": 512, "K": 384, "depth": 0, "tile": 1, "ms": 0.125},\n'
                    '  {"M": 256, "N": 512, "K": 384, "depth": 1, "tile": 0, "ms": 0.250}\n]}\n')
    before = fastmm.planner_records()
    fastmm.planner_load(str(good), None)
    assert fastmm.planner_records() == before + 2
    out = tmp_path / "out.json"
    fastmm.planner_save(str(out), None)
    assert '"M": 256, "N": 512, "K": 384, "depth": 1, "tile": 0, "ms": 0.250000' in out.read_text()
    bad = tmp_path / "bad.json"
    bad.write_text('{"records": [{"M": 256, "N": -5, "K": 384, "depth": 0, "tile": 1, "ms": 1.0}]}')
    with pytest.raises(fastmm.FastmmError) as e:
        fastmm.planner_load(str(bad), None)
    assert e.value.code == fastmm.ERROR_INVALID_VALUE
    assert fastmm.planner_records() == before + 2  # nothing appended on error
    with pytest.raises(fastmm.FastmmError):
        fastmm.planner_load(str(tmp_path / "missing.json"), None)
    with pytest.raises(fastmm.FastmmError):
        fastmm.plan(8, 8, 8, 7)  # unknown mode
