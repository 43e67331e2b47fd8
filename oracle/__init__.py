"""ORACLE -- test infrastructure, not part of the library.

A plain, slow, obviously correct CPU implementation of what the GPU library
computes, written from the paper and from the mathematics.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with ``paper_1205_2927_amd`` (the GPU library)
and never imports it; the only module both sides use is ``synthgen`` (seeded
inputs, no arithmetic of the method).

Contents
  classic   -- c_ij = sum_k a_ik b_kj in FP64/int64 (equation (6)), plus the
               sampled-row and Freivalds helpers for sizes too large for a
               full product.
  winograd  -- Winograd's 7-product variant of Strassen's recursion with the
               paper's quadrant split (equation (1)) and a leaf cutoff; the
               classic 8-product recursion of Table 1 (RMUL); the two-device
               column split of equations (3)-(4); structure counts.
  mlp       -- the planner's cost-model network in FP64: forward, analytic
               backward, Adam.
  checks    -- relative Frobenius error and the probabilistic checks.
  split     -- the precision forms of the leaf (split BF16, scaled split
               FP16) emulated in numpy, and Winograd's recursion over
               them with FP32 additions.
"""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    """Compile ref_gemm.c into liboracle.so (gcc, OpenMP).  Building the
    checker is not using it: the library never loads this file."""
    src = os.path.join(_HERE, "ref_gemm.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", LIB_PATH + ".tmp", src]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


from . import checks, classic, mlp, winograd  # noqa: E402,F401
