"""fastmm for MI355X: FP32 C = A*B by Winograd's variant of Strassen's
recursion with MFMA leaf products (gfx950).

The compute path is the native library ``libfastmm.so`` (hand-written HIP
kernels behind a C ABI, declared in ``include/fastmm.h``); ``fastmm`` is a
thin ctypes binding with the same function names.  PyTorch only supplies
device memory, pinned host memory and streams.
"""
from . import fastmm  # noqa: F401

__all__ = ["fastmm"]
