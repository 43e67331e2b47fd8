"""CPU-side checks of the boundary: the library builds, loads, and exports
every function include/fastmm.h declares.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastmm.h")


def declared_functions():
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fastmm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_three_entry_points():
    names = declared_functions()
    for n in ("fastmm_gemm", "fastmm_gemm_batched", "fastmm_plan"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1205_2927_amd import fastmm
    lib = fastmm.load()
    names = declared_functions()
    assert sorted(fastmm.EXPORTS) == names
    for n in names:
        assert isinstance(getattr(lib, n), ctypes._CFuncPtr)


def test_binding_has_no_cpu_fallback(tmp_path):
    from paper_1205_2927_amd import fastmm
    with pytest.raises(RuntimeError):
        # a fresh loader pointed at a missing file must raise, not fall back
        saved = fastmm._lib
        fastmm._lib = None
        try:
            fastmm.load(str(tmp_path / "missing.so"))
        finally:
            fastmm._lib = saved


def test_struct_layouts_match_header():
    from paper_1205_2927_amd import fastmm
    # fastmm_plan_t: int, int64, int, size_t, double, int -> 48 bytes on LP64
    assert ctypes.sizeof(fastmm.Plan) == 48
    assert ctypes.sizeof(fastmm.Stats) == 4 + 4 + 8 * 4 + 8 * 3 + 4 + 4 + 8 + 8 * 6 + 8


def test_oracle_is_not_linked_by_the_library():
    so = os.path.join(ROOT, "paper_1205_2927_amd", "libfastmm.so")
    with open(so, "rb") as f:
        data = f.read()
    assert b"liboracle" not in data and b"ref_gemm" not in data
    pkg = os.path.join(ROOT, "paper_1205_2927_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                with open(os.path.join(dirpath, f)) as fh:
                    src = fh.read()
                assert "import oracle" not in src and "from oracle" not in src, f
