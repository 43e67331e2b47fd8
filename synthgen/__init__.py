"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the matrix-multiplication method: it only
turns (seed, element index) into numbers.  The paper measures on square
matrices of given sizes and never states the values in them (Section 4,
"Experimental Results": performance is 2N^3 over wall-clock); the inputs used
here are therefore synthetic.

Generator: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), used as a
counter-based generator.  Element ``i`` (0-based, logical row-major index
``r * cols + c``, independent of any leading dimension) of the stream with
seed ``s`` is ``mix(s + (i + 1) * GAMMA)`` -- exactly the ``i``-th output of
the sequential SplitMix64 started from state ``s``.

Value maps (all exactly representable in FP32 and never subnormal):

* ``uniform_pm1``: ``(z >> 40) * 2**-23 - 1``, a 2**-23 grid on [-1, 1).
* ``int_range(lo, hi)``: ``lo + (z >> 32) % (hi - lo + 1)``, small integers.
* ``loguniform``: ``x = +-(1 + f) * 2**E`` with the octave ``E`` uniform over
  the integers ``emin .. emax-1`` (from ``(z >> 32) % (emax - emin)``), the
  mantissa fraction ``f`` on the 2**-23 grid of [0, 1) (bits 8..30 of ``z``)
  and the sign from bit 0: magnitudes spread evenly over the octaves
  2**emin .. 2**emax, exactly representable, identical in C and numpy.

A C implementation of the same maps (``gen.c``) fills large host buffers with
OpenMP; ``tests/test_synthgen.py`` checks that it agrees bit-for-bit with the
numpy definition below.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynthgen.so")
_lib = None


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function (the 'mix64' finaliser) on uint64 arrays."""
    z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


def stream(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs ``start .. start+count-1`` of SplitMix64 started from ``seed``."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        state = np.uint64(seed % 2**64) + idx * np.uint64(GAMMA)
        return _mix(state)


def _to_uniform_pm1(z: np.ndarray) -> np.ndarray:
    k = (z >> np.uint64(40)).astype(np.int64)  # 0 .. 2**24-1
    return ((k - (1 << 23)).astype(np.float64) * 2.0**-23).astype(np.float32)


def uniform_pm1_np(seed: int, rows: int, cols: int) -> np.ndarray:
    """rows x cols float32 matrix, entries on the 2**-23 grid of [-1, 1)."""
    return _to_uniform_pm1(stream(seed, 0, rows * cols)).reshape(rows, cols)


def int_range_np(seed: int, rows: int, cols: int, lo: int, hi: int) -> np.ndarray:
    """rows x cols float32 matrix of integers in [lo, hi]."""
    z = stream(seed, 0, rows * cols)
    span = np.uint64(hi - lo + 1)
    v = ((z >> np.uint64(32)) % span).astype(np.int64) + lo
    return v.astype(np.float32).reshape(rows, cols)


def loguniform_np(seed: int, rows: int, cols: int, emin: int = -8,
                  emax: int = 8) -> np.ndarray:
    """rows x cols float32 matrix, |x| spread evenly over octaves [2**emin, 2**emax)."""
    z = stream(seed, 0, rows * cols)
    octave = ((z >> np.uint64(32)) % np.uint64(emax - emin)).astype(np.int64) + emin
    frac = ((z >> np.uint64(8)) & np.uint64((1 << 23) - 1)).astype(np.float64) * 2.0**-23
    sign = np.where((z & np.uint64(1)) == 1, -1.0, 1.0)
    return (sign * np.ldexp(1.0 + frac, octave)).astype(np.float32).reshape(rows, cols)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            return None
        lib = ctypes.CDLL(_LIB_PATH)
        u64, i64, i32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32
        vp = ctypes.c_void_p
        lib.synth_uniform_pm1_f32.argtypes = [u64, i64, i64, i64, vp]
        lib.synth_int_range_f32.argtypes = [u64, i64, i64, i64, i32, i32, vp]
        lib.synth_loguniform_f32.argtypes = [u64, i64, i64, i64, i32, i32, vp]
        for f in (lib.synth_uniform_pm1_f32, lib.synth_int_range_f32,
                  lib.synth_loguniform_f32):
            f.restype = None
        _lib = lib
    return _lib


def build(verbose: bool = False) -> str:
    """Compile gen.c into libsynthgen.so next to this file (gcc + OpenMP)."""
    import subprocess
    src = os.path.join(_HERE, "gen.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", _LIB_PATH + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def fill_uniform_pm1(seed: int, rows: int, cols: int, ptr: int, ld: int | None = None) -> None:
    """Fill a host buffer at address ``ptr`` (row-major, leading dim ``ld``)."""
    lib = _load()
    if lib is None:
        raise RuntimeError("libsynthgen.so is not built; call synthgen.build()")
    lib.synth_uniform_pm1_f32(seed, rows, cols, cols if ld is None else ld, ptr)


def fill_int_range(seed: int, rows: int, cols: int, lo: int, hi: int, ptr: int,
                   ld: int | None = None) -> None:
    lib = _load()
    if lib is None:
        raise RuntimeError("libsynthgen.so is not built; call synthgen.build()")
    lib.synth_int_range_f32(seed, rows, cols, cols if ld is None else ld, lo, hi, ptr)


def fill_loguniform(seed: int, rows: int, cols: int, ptr: int, ld: int | None = None,
                    emin: int = -8, emax: int = 8) -> None:
    lib = _load()
    if lib is None:
        raise RuntimeError("libsynthgen.so is not built; call synthgen.build()")
    lib.synth_loguniform_f32(seed, rows, cols, cols if ld is None else ld, emin, emax, ptr)


def uniform_pm1(seed: int, rows: int, cols: int) -> np.ndarray:
    """Same values as ``uniform_pm1_np``; uses the C filler when it is built."""
    if _load() is None or rows * cols < (1 << 16):
        return uniform_pm1_np(seed, rows, cols)
    out = np.empty((rows, cols), dtype=np.float32)
    fill_uniform_pm1(seed, rows, cols, out.ctypes.data)
    return out


def int_range(seed: int, rows: int, cols: int, lo: int, hi: int) -> np.ndarray:
    if _load() is None or rows * cols < (1 << 16):
        return int_range_np(seed, rows, cols, lo, hi)
    out = np.empty((rows, cols), dtype=np.float32)
    fill_int_range(seed, rows, cols, lo, hi, out.ctypes.data)
    return out


def loguniform(seed: int, rows: int, cols: int, emin: int = -8,
               emax: int = 8) -> np.ndarray:
    if _load() is None or rows * cols < (1 << 16):
        return loguniform_np(seed, rows, cols, emin, emax)
    out = np.empty((rows, cols), dtype=np.float32)
    fill_loguniform(seed, rows, cols, out.ctypes.data, emin=emin, emax=emax)
    return out


def shapes_loguniform(seed: int, count: int, lo: int = 256, hi: int = 6144,
                      multiple: int = 64) -> np.ndarray:
    """``count`` x 3 int64 array of (M, N, K), each log-uniform in [lo, hi] and
    rounded to a multiple of ``multiple`` (clamped into [lo, hi])."""
    z = stream(seed, 0, 3 * count)
    u = (z >> np.uint64(11)).astype(np.float64) * 2.0**-53
    v = np.exp(np.log(lo) + (np.log(hi) - np.log(lo)) * u)
    r = np.rint(v / multiple).astype(np.int64) * multiple
    r = np.clip(r, lo, hi)
    return r.reshape(count, 3)


def batch_seeds(config: int, i: int) -> tuple[int, int]:
    """Seeds of the A and B operands of problem ``i`` of a batched workload
    of configuration ``config``: (1001 + config) * 1000 + i and
    (2001 + config) * 1000 + i (disjoint for i < 1000)."""
    if not 0 <= i < 1000:
        raise ValueError("problem index out of range")
    return (1001 + config) * 1000 + i, (2001 + config) * 1000 + i


def signs_pm1(seed: int, count: int) -> np.ndarray:
    """``count`` values in {-1.0, +1.0} (float64), from bit 63 of the stream."""
    z = stream(seed, 0, count)
    return np.where((z >> np.uint64(63)) == 1, -1.0, 1.0)


def row_sample(seed: int, n_rows: int, count: int) -> np.ndarray:
    """``count`` distinct row indices in [0, n_rows), sorted (seeded)."""
    count = min(count, n_rows)
    z = stream(seed, 0, n_rows)
    order = np.argsort(z, kind="stable")
    return np.sort(order[:count]).astype(np.int64)
