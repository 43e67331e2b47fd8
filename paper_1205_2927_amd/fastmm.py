"""ctypes binding of libfastmm.so (argument marshalling only).

Every function mirrors an entry point of ``include/fastmm.h`` under the same
name without the ``fastmm_`` prefix.  Matrix arguments may be torch tensors
(device or host, FP32, row-major with unit column stride) or raw integer
addresses with explicit leading dimensions.  A non-zero status raises
``FastmmError`` carrying the library's message.  There is no fallback: if the
library is not built, ``load()`` raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfastmm.so")

SUCCESS = 0
ERROR_INVALID_VALUE = -1
ERROR_OUT_OF_MEMORY = -2
ERROR_DEVICE = -3
ERROR_NOT_SUPPORTED = -4

AUTO = -1
PLAN_DEFAULT, PLAN_MODEL, PLAN_EXHAUSTIVE = 0, 1, 2
TILE_128x128, TILE_256x128, TILE_128x64, TILE_64x64 = 0, 1, 2, 3
TILE_128x128_K32, TILE_256x128_W8, TILE_256x256_W8, TILE_128x256 = 4, 5, 6, 7
TILE_BF16X3 = 8  # split-BF16 precision form of the leaf (256x256 tiles on packed operands)
TILE_FP16X3 = 9  # scaled split-FP16 precision form of the leaf (256x256 tiles on packed operands)
TILES = {TILE_128x128: (128, 128), TILE_256x128: (256, 128), TILE_128x64: (128, 64),
         TILE_64x64: (64, 64), TILE_128x128_K32: (128, 128), TILE_256x128_W8: (256, 128),
         TILE_256x256_W8: (256, 256), TILE_128x256: (128, 256), TILE_BF16X3: (256, 256),
         TILE_FP16X3: (256, 256)}
MLP_PARAMS = 4609
MODEL_NETS = 3  # networks of the planner's cost model (model file: MODEL_NETS x MLP_PARAMS floats)

# Every symbol include/fastmm.h declares.
EXPORTS = [
    "fastmm_gemm", "fastmm_gemm_ex", "fastmm_rmul", "fastmm_gemm_batched", "fastmm_plan",
    "fastmm_set_plan_mode", "fastmm_planner_load", "fastmm_planner_save",
    "fastmm_planner_train", "fastmm_planner_records", "fastmm_set_stream",
    "fastmm_set_profiling", "fastmm_get_stats", "fastmm_get_last_error", "fastmm_finalize",
    "fastmm_preadd", "fastmm_postadd", "fastmm_mlp_forward", "fastmm_mlp_backward",
    "fastmm_mlp_adam", "fastmm_gemm_noalloc",
]
NOALLOC_WORKSPACE_BYTES = 256 << 20


class FastmmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fastmm error {code}: {msg}")
        self.code = code


class Plan(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int), ("leaf", ctypes.c_int64), ("tile", ctypes.c_int),
                ("workspace_bytes", ctypes.c_size_t), ("predicted_ms", ctypes.c_double),
                ("source", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int), ("tile", ctypes.c_int), ("leaves", ctypes.c_int64),
                ("leaf_m", ctypes.c_int64), ("leaf_k", ctypes.c_int64), ("leaf_n", ctypes.c_int64),
                ("leaf_flops", ctypes.c_double), ("add_bytes", ctypes.c_double),
                ("transfer_bytes", ctypes.c_double), ("launches", ctypes.c_int),
                ("workspace_bytes", ctypes.c_size_t), ("h2d_ms", ctypes.c_double),
                ("preadd_ms", ctypes.c_double), ("leaf_ms", ctypes.c_double),
                ("postadd_ms", ctypes.c_double), ("d2h_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("leaf_launches", ctypes.c_int),
                ("graph_replayed", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def load(path: str | None = None):
    """Load libfastmm.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1205_2927_amd.build`")
    # torch ships its own HIP runtime under the same soname; loading torch
    # first makes the library bind to that one runtime instead of bringing a
    # second copy into the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    i64, i32, vp, f32 = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_float
    P64 = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "fastmm_gemm": [i64, i64, i64, vp, i64, vp, i64, vp, i64, i32, i64],
        "fastmm_gemm_ex": [i64, i64, i64, vp, i64, vp, i64, vp, i64, i32, i64, i32],
        "fastmm_gemm_noalloc": [i64, i64, i64, vp, i64, vp, i64, vp, i64, i32, i64],
        "fastmm_rmul": [i64, i64, i64, vp, i64, vp, i64, vp, i64, i32, i64, i32],
        "fastmm_gemm_batched": [i32, P64, P64, P64, vp, P64, vp, P64, vp, P64, vp, vp],
        "fastmm_plan": [i64, i64, i64, i32, ctypes.POINTER(Plan)],
        "fastmm_set_plan_mode": [i32],
        "fastmm_planner_load": [ctypes.c_char_p, ctypes.c_char_p],
        "fastmm_planner_save": [ctypes.c_char_p, ctypes.c_char_p],
        "fastmm_planner_train": [i32, i32, f32, ctypes.c_uint64, ctypes.POINTER(f32)],
        "fastmm_planner_records": [],
        "fastmm_set_stream": [vp],
        "fastmm_set_profiling": [i32],
        "fastmm_get_stats": [ctypes.POINTER(Stats)],
        "fastmm_get_last_error": [],
        "fastmm_finalize": [],
        "fastmm_preadd": [i32, i64, i64, vp, i64, vp],
        "fastmm_postadd": [i64, i64, vp, vp, i64, i64, i64],
        "fastmm_mlp_forward": [i32, vp, vp, vp],
        "fastmm_mlp_backward": [i32, vp, vp, vp, vp, vp],
        "fastmm_mlp_adam": [vp, vp, vp, vp, i32, f32, f32, f32, f32],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.fastmm_get_last_error.restype = ctypes.c_char_p
    lib.fastmm_finalize.restype = None
    lib.fastmm_planner_records.restype = ctypes.c_int64
    _lib = lib
    return lib


def last_error() -> str:
    return load().fastmm_get_last_error().decode()


def _check(rc: int):
    if rc != SUCCESS:
        raise FastmmError(rc, last_error())


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _ld(x, ld):
    if ld is not None:
        return int(ld)
    if x is None or isinstance(x, int):
        raise ValueError("leading dimension required for raw pointers")
    if x.dim() != 2 or x.stride(1) != 1:
        raise ValueError("expected a 2-D row-major tensor with unit column stride")
    return max(1, int(x.stride(0)))


def gemm(M, N, K, A, B, C, depth=0, leaf=1280, tile=None, lda=None, ldb=None, ldc=None):
    """fastmm_gemm / fastmm_gemm_ex: C = A B.  Returns the status (raises on error)."""
    lib = load()
    if tile is None:
        rc = lib.fastmm_gemm(M, N, K, _ptr(A), _ld(A, lda), _ptr(B), _ld(B, ldb), _ptr(C),
                             _ld(C, ldc), int(depth), int(leaf))
    else:
        rc = lib.fastmm_gemm_ex(M, N, K, _ptr(A), _ld(A, lda), _ptr(B), _ld(B, ldb), _ptr(C),
                                _ld(C, ldc), int(depth), int(leaf), int(tile))
    _check(rc)
    return rc


def gemm_noalloc(M, N, K, A, B, C, depth=0, leaf=1280, lda=None, ldb=None, ldc=None):
    """fastmm_gemm_noalloc: C = A B in the library's static device workspace."""
    _check(load().fastmm_gemm_noalloc(M, N, K, _ptr(A), _ld(A, lda), _ptr(B), _ld(B, ldb),
                                      _ptr(C), _ld(C, ldc), int(depth), int(leaf)))


def gemm_noalloc_raw(M, N, K, A, lda, B, ldb, C, ldc, depth, leaf) -> int:
    """Status code of fastmm_gemm_noalloc without raising."""
    return load().fastmm_gemm_noalloc(M, N, K, A, lda, B, ldb, C, ldc, depth, leaf)


def rmul(M, N, K, A, B, C, depth=0, leaf=3008, tile=TILE_128x128, lda=None, ldb=None, ldc=None):
    """fastmm_rmul: C = A B by the classic 8-product recursion (comparator)."""
    _check(load().fastmm_rmul(M, N, K, _ptr(A), _ld(A, lda), _ptr(B), _ld(B, ldb), _ptr(C),
                              _ld(C, ldc), int(depth), int(leaf), int(tile)))


def gemm_raw(M, N, K, A, lda, B, ldb, C, ldc, depth, leaf, tile=None) -> int:
    """Status code without raising (for error-path tests)."""
    lib = load()
    if tile is None:
        return lib.fastmm_gemm(M, N, K, A, lda, B, ldb, C, ldc, depth, leaf)
    return lib.fastmm_gemm_ex(M, N, K, A, lda, B, ldb, C, ldc, depth, leaf, tile)


def matmul(A, B, depth=0, leaf=1280, tile=None, out=None):
    """Convenience: C = A @ B for 2-D FP32 tensors (same residency)."""
    import torch
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    C = out if out is not None else torch.empty((M, N), dtype=torch.float32, device=A.device,
                                                 pin_memory=(A.device.type == "cpu" and A.is_pinned()))
    gemm(M, N, K, A, B, C, depth=depth, leaf=leaf, tile=tile)
    return C


def gemm_batched(As, Bs, Cs, depth=None, leaf=None, check=True):
    """fastmm_gemm_batched over lists of 2-D tensors."""
    lib = load()
    n = len(As)
    I64 = ctypes.c_int64 * n
    VP = ctypes.c_void_p * n
    M = I64(*[a.shape[0] for a in As])
    K = I64(*[a.shape[1] for a in As])
    N = I64(*[b.shape[1] for b in Bs])
    lda = I64(*[_ld(a, None) for a in As])
    ldb = I64(*[_ld(b, None) for b in Bs])
    ldc = I64(*[_ld(c, None) for c in Cs])
    pa = VP(*[_ptr(a) for a in As])
    pb = VP(*[_ptr(b) for b in Bs])
    pc = VP(*[_ptr(c) for c in Cs])
    dep = (ctypes.c_int * n)(*depth) if depth is not None else None
    lf = I64(*leaf) if leaf is not None else None
    rc = lib.fastmm_gemm_batched(n, M, N, K, pa, lda, pb, ldb, pc, ldc,
                                 ctypes.cast(dep, ctypes.c_void_p) if dep is not None else None,
                                 ctypes.cast(lf, ctypes.c_void_p) if lf is not None else None)
    if check:
        _check(rc)
    return rc


class Batch:
    """fastmm_gemm_batched over fixed lists of 2-D tensors, its argument
    arrays built once: each call passes them again as they are (for
    repeated products on the same buffers, e.g. a serving loop; building
    the arrays for 256 problems costs about a millisecond of Python per
    call).  The tensors are kept alive by the object."""

    def __init__(self, As, Bs, Cs, depth=None, leaf=None):
        n = len(As)
        I64 = ctypes.c_int64 * n
        VP = ctypes.c_void_p * n
        self._keep = (list(As), list(Bs), list(Cs))
        self._n = n
        self._M = I64(*[a.shape[0] for a in As])
        self._K = I64(*[a.shape[1] for a in As])
        self._N = I64(*[b.shape[1] for b in Bs])
        self._lda = I64(*[_ld(a, None) for a in As])
        self._ldb = I64(*[_ld(b, None) for b in Bs])
        self._ldc = I64(*[_ld(c, None) for c in Cs])
        self._pa = VP(*[_ptr(a) for a in As])
        self._pb = VP(*[_ptr(b) for b in Bs])
        self._pc = VP(*[_ptr(c) for c in Cs])
        self._dep = (ctypes.c_int * n)(*depth) if depth is not None else None
        self._lf = I64(*leaf) if leaf is not None else None
        self._depp = ctypes.cast(self._dep, ctypes.c_void_p) if self._dep is not None else None
        self._lfp = ctypes.cast(self._lf, ctypes.c_void_p) if self._lf is not None else None

    def __call__(self, check=True):
        rc = load().fastmm_gemm_batched(self._n, self._M, self._N, self._K, self._pa, self._lda,
                                        self._pb, self._ldb, self._pc, self._ldc, self._depp, self._lfp)
        if check:
            _check(rc)
        return rc


def gemm_batched_raw(M, N, K, A, lda, B, ldb, C, ldc, depth=None, leaf=None) -> int:
    """fastmm_gemm_batched on plain lists of extents, addresses and leading
    dimensions; returns the status without raising (for error-path tests)."""
    lib = load()
    n = len(M)
    I64 = ctypes.c_int64 * n
    VP = ctypes.c_void_p * n
    dep = (ctypes.c_int * n)(*depth) if depth is not None else None
    lf = I64(*leaf) if leaf is not None else None
    return lib.fastmm_gemm_batched(n, I64(*M), I64(*N), I64(*K), VP(*A), I64(*lda), VP(*B),
                                   I64(*ldb), VP(*C), I64(*ldc),
                                   ctypes.cast(dep, ctypes.c_void_p) if dep is not None else None,
                                   ctypes.cast(lf, ctypes.c_void_p) if lf is not None else None)


def plan(M, N, K, mode=PLAN_DEFAULT) -> Plan:
    p = Plan()
    _check(load().fastmm_plan(M, N, K, mode, ctypes.byref(p)))
    return p


def set_plan_mode(mode: int):
    _check(load().fastmm_set_plan_mode(mode))


def planner_load(db_path=None, model_path=None):
    _check(load().fastmm_planner_load(db_path.encode() if db_path else None,
                                      model_path.encode() if model_path else None))


def planner_save(db_path=None, model_path=None):
    _check(load().fastmm_planner_save(db_path.encode() if db_path else None,
                                      model_path.encode() if model_path else None))


def planner_train(epochs=200, batch=64, lr=1e-3, seed=4001) -> float:
    loss = ctypes.c_float(0.0)
    _check(load().fastmm_planner_train(epochs, batch, lr, seed, ctypes.byref(loss)))
    return float(loss.value)


def planner_records() -> int:
    return int(load().fastmm_planner_records())


def set_stream(stream=None):
    """stream: a torch.cuda.Stream, a raw hipStream_t address, or None."""
    handle = 0 if stream is None else (stream if isinstance(stream, int) else stream.cuda_stream)
    _check(load().fastmm_set_stream(handle or None))


def set_profiling(on: bool):
    _check(load().fastmm_set_profiling(1 if on else 0))


def get_stats() -> dict:
    s = Stats()
    _check(load().fastmm_get_stats(ctypes.byref(s)))
    return s.as_dict()


def finalize():
    load().fastmm_finalize()


def preadd(side, rows, cols, X, out, ldx=None):
    _check(load().fastmm_preadd(side, rows, cols, _ptr(X), _ld(X, ldx), _ptr(out)))


def postadd(h_r, h_c, P, C, rows, cols, ldc=None):
    _check(load().fastmm_postadd(h_r, h_c, _ptr(P), _ptr(C), _ld(C, ldc), rows, cols))


def mlp_forward(batch, params, X, y):
    _check(load().fastmm_mlp_forward(batch, _ptr(params), _ptr(X), _ptr(y)))


def mlp_backward(batch, params, X, t, grad, loss=None):
    _check(load().fastmm_mlp_backward(batch, _ptr(params), _ptr(X), _ptr(t), _ptr(grad),
                                      _ptr(loss) if loss is not None else None))


def mlp_adam(grad, params, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(load().fastmm_mlp_adam(_ptr(grad), _ptr(params), _ptr(m), _ptr(v), step, lr, beta1,
                                  beta2, eps))
