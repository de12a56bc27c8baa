"""Python binding of libflyte (the C ABI of ``include/flyte.h``).

Argument marshalling only: every operation runs in the HIP kernels of
``libflyte.so``.  PyTorch supplies device memory (packed arrays are ``uint8``
tensors of n*k bytes) and the current stream.  If the library is missing it is
built with hipcc; if that fails, every call raises -- there is no CPU path.
"""
from __future__ import annotations

import ctypes
import os
import threading
from dataclasses import dataclass

import torch

from . import build as _build

FORMATS = [(32, 2), (32, 3), (32, 4)] + [(64, k) for k in range(2, 9)]

FB_OK, FB_ERR_FORMAT, FB_ERR_ARG, FB_ERR_ALIGN, FB_ERR_UNSUPPORTED, FB_ERR_RUNTIME = range(6)


class FlyteError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{status_name(status)}: {detail}")
        self.status = status


ROUND_NEAREST_EVEN, ROUND_TOWARD_ZERO, ROUND_TO_ODD = 0, 1, 2


class fb_format(ctypes.Structure):
    _fields_ = [("base", ctypes.c_uint8), ("k", ctypes.c_uint8), ("round", ctypes.c_uint8),
                ("reserved", ctypes.c_uint8)]


class fb_gemv_desc(ctypes.Structure):
    _fields_ = [("f", fb_format), ("m", ctypes.c_int32),
                ("n", ctypes.c_int32), ("reserved1", ctypes.c_int32), ("lda", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("x", ctypes.c_void_p), ("y", ctypes.c_void_p)]


assert ctypes.sizeof(fb_gemv_desc) == 48

_lock = threading.Lock()
_lib = None

_P, _I32, _I64, _SZ, _DBL = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
_SIGS = {
    "fb_pack": (_I32, [fb_format, _P, _P, _SZ, _P]),
    "fb_unpack": (_I32, [fb_format, _P, _P, _SZ, _P]),
    "fb_dot": (_I32, [fb_format, _SZ, _P, _P, _P, _P]),
    "fb_dot_noalloc": (_I32, [fb_format, _SZ, _P, _P, _P, _P]),
    "fb_axpy": (_I32, [fb_format, _SZ, _DBL, _P, _P, _P]),
    "fb_scale": (_I32, [fb_format, _SZ, _DBL, _P, _P]),
    "fb_nrm2": (_I32, [fb_format, _SZ, _P, _P, _P]),
    "fb_gemv": (_I32, [fb_format, _I64, _I64, _P, _I64, _P, _P, _P]),
    "fb_gemv_config": (_I32, [fb_format, _I64, _I64, _P, _I64, _P, _P, _I32, _P]),
    "fb_gemv_ex": (_I32, [fb_format, fb_format, _I32, _I64, _I64, _P, _I64, _P, _P, _P]),
    "fb_dot_packed": (_I32, [fb_format, fb_format, _SZ, _P, _P, _P, _P]),
    "fb_gemv_num_configs": (_I32, []),
    "fb_gemv_config_info": (_I32, [_I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
    "fb_tune_gemv": (_I32, [fb_format, _I64, _I64, _P, _I64, _P, _P, _I32, ctypes.POINTER(_I32), _P]),
    "fb_tune_lookup": (_I32, [fb_format, _I64, _I64]),
    "fb_tune_record": (_I32, [fb_format, _I64, _I64, _I32, _DBL]),
    "fb_tune_save": (_I32, [ctypes.c_char_p]),
    "fb_tune_load": (_I32, [ctypes.c_char_p]),
    "fb_tune_clear": (None, []),
    "fb_gemv_batched_plan": (_I32, [ctypes.POINTER(fb_gemv_desc), _I32, ctypes.POINTER(_P)]),
    "fb_gemv_batched_tune": (_I32, [_P, _I32, _P]),
    "fb_gemv_batched_launch": (_I32, [_P, _P]),
    "fb_gemv_batched_loop": (_I32, [_P, _P]),
    "fb_gemv_batched_loop_graph": (_I32, [_P, _P]),
    "fb_plan_bytes": (_I64, [_P]),
    "fb_plan_config": (_I32, [_P, _I32]),
    "fb_plan_destroy": (None, [_P]),
    "fb_gemm": (_I32, [fb_format, fb_format, fb_format, _I64, _I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P]),
    "fb_gemm_ex": (_I32, [fb_format, fb_format, fb_format, _I64, _I64, _I64, _P, _I64, _P, _I64, _P, _I64,
                          ctypes.c_uint32, _P]),
    "fb_status_str": (ctypes.c_char_p, [_I32]),
    "fb_last_error": (ctypes.c_char_p, []),
}


def lib_path() -> str:
    return _build.LIB


def load() -> ctypes.CDLL:
    """Loads libflyte.so (building it first if it is absent)."""
    global _lib
    with _lock:
        if _lib is None:
            path = lib_path()
            if not os.path.exists(path):
                _build.build()
            if not os.path.exists(path):
                raise RuntimeError(f"libflyte.so is missing at {path} and could not be built")
            lib = ctypes.CDLL(path)
            for name, (res, args) in _SIGS.items():
                fn = getattr(lib, name, None)
                if fn is None:
                    continue
                fn.restype = res
                fn.argtypes = args
            _lib = lib
        return _lib


def status_name(status: int) -> str:
    return load().fb_status_str(status).decode()


def last_error() -> str:
    return load().fb_last_error().decode()


def _check(status: int) -> None:
    if status != FB_OK:
        raise FlyteError(status, last_error())


def fmt(f) -> fb_format:
    """(base, k) or (base, k, round) -> fb_format."""
    if isinstance(f, fb_format):
        return f
    base, k = f[0], f[1]
    return fb_format(base, k, f[2] if len(f) > 2 else 0, 0)


def native_dtype(base: int) -> torch.dtype:
    return torch.float32 if base == 32 else torch.float64


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _arg(t, name: str, nbytes: int, dtype: torch.dtype | None = None, like: torch.Tensor | None = None) -> int:
    """Checks a tensor handed to the library and returns its device address.

    The kernels read and write raw device memory through the pointer, so a
    host tensor, a strided view or a buffer smaller than the call touches
    would be an out-of-bounds device access; each is refused here instead.
    dtype None accepts any element type (packed bytes may be viewed as
    anything); otherwise the tensor must have that dtype."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise ValueError(f"{name}: tensor is on {t.device}, the library needs device memory")
    if like is not None and t.device != like.device:
        raise ValueError(f"{name}: tensor is on {t.device}, the call's other operands on {like.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name}: expected dtype {dtype}, got {t.dtype}")
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise ValueError(f"{name}: the call touches {nbytes} bytes, the tensor holds {have}")
    return t.data_ptr()


def _out_dtype(base: int, k: int) -> torch.dtype:
    """Element type of an output in format (base, k): native when k is the base width, else bytes."""
    return native_dtype(base) if 8 * k == base else torch.uint8


def _mat_bytes(rows: int, cols: int, ld: int, elem: int) -> int:
    """Bytes spanned by a rows x cols row-major matrix with leading dimension ld."""
    if rows <= 0 or cols <= 0:
        return 0
    return ((rows - 1) * ld + cols) * elem


# ---------------------------------------------------------------- codec
def pack(f, src: torch.Tensor, out: torch.Tensor | None = None, n: int | None = None, stream=None):
    """Rounds native values (float32 for base 32, float64 for base 64) to k-byte elements
    (f = (base, k) or (base, k, round))."""
    base, k = f[0], f[1]
    n = src.numel() if n is None else n
    if out is None:
        out = torch.empty(n * k, dtype=torch.uint8, device=src.device)
    ps = _arg(src, "pack: src", n * base // 8, native_dtype(base))
    po = _arg(out, "pack: out", n * k, None, src)
    _check(load().fb_pack(fmt(f), ps, po, n, _stream(stream)))
    return out


def unpack(f, packed: torch.Tensor, n: int | None = None, out: torch.Tensor | None = None, stream=None):
    base, k = f[0], f[1]
    n = packed.numel() // k if n is None else n
    if out is None:
        out = torch.empty(n, dtype=native_dtype(base), device=packed.device)
    pp = _arg(packed, "unpack: packed", n * k)
    po = _arg(out, "unpack: out", n * base // 8, native_dtype(base), packed)
    _check(load().fb_unpack(fmt(f), pp, po, n, _stream(stream)))
    return out


# ---------------------------------------------------------------- BLAS 1
def dot(f, x: torch.Tensor, y: torch.Tensor, n: int | None = None, out: torch.Tensor | None = None, stream=None):
    base, k = f[0], f[1]
    n = x.numel() // k if n is None else n
    if out is None:
        out = torch.empty((), dtype=native_dtype(base), device=x.device)
    px = _arg(x, "dot: x", n * k)
    py = _arg(y, "dot: y", n * k, None, x)
    po = _arg(out, "dot: out", base // 8, native_dtype(base), x)
    _check(load().fb_dot(fmt(f), n, px, py, po, _stream(stream)))
    return out


def dot_noalloc(f, x: torch.Tensor, y: torch.Tensor, out: torch.Tensor, n: int | None = None, stream=None):
    """dot through the allocation-free entry point (partial sums in a static device
    array shared by every call on the device; out must be given)."""
    base, k = f[0], f[1]
    n = x.numel() // k if n is None else n
    px = _arg(x, "dot_noalloc: x", n * k)
    py = _arg(y, "dot_noalloc: y", n * k, None, x)
    po = _arg(out, "dot_noalloc: out", base // 8, native_dtype(base), x)
    _check(load().fb_dot_noalloc(fmt(f), n, px, py, po, _stream(stream)))
    return out


def axpy(f, alpha: float, x: torch.Tensor, y: torch.Tensor, n: int | None = None, stream=None):
    """y <- pack(alpha * x + y), in place on the packed tensor y."""
    base, k = f[0], f[1]
    n = y.numel() // k if n is None else n
    py = _arg(y, "axpy: y", n * k)
    px = _arg(x, "axpy: x", n * k, None, y)
    _check(load().fb_axpy(fmt(f), n, float(alpha), px, py, _stream(stream)))
    return y


def scale(f, alpha: float, x: torch.Tensor, n: int | None = None, stream=None):
    """x <- pack(alpha * x), in place on the packed tensor x."""
    base, k = f[0], f[1]
    n = x.numel() // k if n is None else n
    px = _arg(x, "scale: x", n * k)
    _check(load().fb_scale(fmt(f), n, float(alpha), px, _stream(stream)))
    return x


def nrm2(f, x: torch.Tensor, n: int | None = None, out: torch.Tensor | None = None, stream=None):
    """sqrt(sum x_i^2) of a packed vector, as a 0-d native tensor on the device."""
    base, k = f[0], f[1]
    n = x.numel() // k if n is None else n
    if out is None:
        out = torch.empty((), dtype=native_dtype(base), device=x.device)
    px = _arg(x, "nrm2: x", n * k)
    po = _arg(out, "nrm2: out", base // 8, native_dtype(base), x)
    _check(load().fb_nrm2(fmt(f), n, px, po, _stream(stream)))
    return out


# ---------------------------------------------------------------- BLAS 2
def _gemv_args(what, base, k, m, n, lda, A, x, y, ydtype, ybytes, trans=False):
    """Checks A (m x n, leading dimension lda), x and y of a GEMV; returns their addresses."""
    nx, ny = (m, n) if trans else (n, m)
    if m > 0 and lda < n:
        raise ValueError(f"{what}: lda {lda} < n {n}")
    pa = _arg(A, f"{what}: A", _mat_bytes(m, n, lda, k))
    # with no outputs nothing is read
    px = _arg(x, f"{what}: x", nx * base // 8 if ny > 0 else 0, native_dtype(base), A)
    py = _arg(y, f"{what}: y", ny * ybytes, ydtype, A)
    return pa, px, py


def gemv(f, A: torch.Tensor, m: int, n: int, x: torch.Tensor, y: torch.Tensor | None = None,
         lda: int | None = None, config: int | None = None, stream=None):
    base, k = f[0], f[1]
    lda = n if lda is None else lda
    if y is None:
        y = torch.empty(m, dtype=native_dtype(base), device=A.device)
    pa, px, py = _gemv_args("gemv", base, k, m, n, lda, A, x, y, native_dtype(base), base // 8)
    if config is None:
        _check(load().fb_gemv(fmt(f), m, n, pa, lda, px, py, _stream(stream)))
    else:
        _check(load().fb_gemv_config(fmt(f), m, n, pa, lda, px, py, config, _stream(stream)))
    return y


def gemv_ex(fa, fy, trans: bool, A: torch.Tensor, m: int, n: int, x: torch.Tensor,
            y: torch.Tensor | None = None, lda: int | None = None, stream=None):
    """y = A x (trans False, m outputs) or A^T x (trans True, n outputs), y in format fy."""
    base = fa[0]
    lda = n if lda is None else lda
    ny = n if trans else m
    if y is None:
        if fy[1] * 8 == base:
            y = torch.empty(ny, dtype=native_dtype(base), device=A.device)
        else:
            y = torch.empty(ny * fy[1], dtype=torch.uint8, device=A.device)
    pa, px, py = _gemv_args("gemv_ex", base, fa[1], m, n, lda, A, x, y, _out_dtype(base, fy[1]), fy[1], trans)
    _check(load().fb_gemv_ex(fmt(fa), fmt(fy), 1 if trans else 0, m, n, pa, lda, px, py, _stream(stream)))
    return y


def dot_packed(f, fr, x: torch.Tensor, y: torch.Tensor, n: int | None = None, out: torch.Tensor | None = None,
               stream=None):
    """dot with the result packed in format fr: a uint8 tensor of fr.k bytes."""
    n = x.numel() // f[1] if n is None else n
    if out is None:
        out = torch.empty(fr[1], dtype=torch.uint8, device=x.device)
    px = _arg(x, "dot_packed: x", n * f[1])
    py = _arg(y, "dot_packed: y", n * f[1], None, x)
    po = _arg(out, "dot_packed: out", fr[1], None, x)
    _check(load().fb_dot_packed(fmt(f), fmt(fr), n, px, py, po, _stream(stream)))
    return out


def gemv_num_configs() -> int:
    return load().fb_gemv_num_configs()


def gemv_config_info(config: int):
    rpw, wpb, cpl = _I32(), _I32(), _I32()
    lpr = load().fb_gemv_config_info(config, ctypes.byref(rpw), ctypes.byref(wpb), ctypes.byref(cpl))
    return {"lanes_per_row": lpr, "rows_per_wave": rpw.value, "waves_per_row_group": wpb.value,
            "units_per_lane": cpl.value}


def tune_gemv(f, A, m, n, x, y, lda=None, reps: int = 10, stream=None) -> int:
    lda = n if lda is None else lda
    best = _I32(-1)
    pa, px, py = _gemv_args("tune_gemv", f[0], f[1], m, n, lda, A, x, y, native_dtype(f[0]), f[0] // 8)
    _check(load().fb_tune_gemv(fmt(f), m, n, pa, lda, px, py, reps, ctypes.byref(best), _stream(stream)))
    return best.value


def tune_lookup(f, m, n) -> int:
    return load().fb_tune_lookup(fmt(f), m, n)


def tune_record(f, m, n, config: int, us: float) -> None:
    _check(load().fb_tune_record(fmt(f), m, n, config, float(us)))


def tune_save(path: str) -> None:
    _check(load().fb_tune_save(path.encode()))


def tune_load(path: str) -> None:
    _check(load().fb_tune_load(path.encode()))


def tune_clear() -> None:
    load().fb_tune_clear()


# ---------------------------------------------------------------- batched GEMV
@dataclass
class GemvItem:
    f: tuple
    m: int
    n: int
    lda: int
    A: torch.Tensor
    x: torch.Tensor
    y: torch.Tensor


class BatchedGemv:
    """A plan for many independent GEMVs run by one persistent kernel."""

    def __init__(self, items: list[GemvItem]):
        self.items = items               # keeps the tensors alive
        arr = (fb_gemv_desc * max(1, len(items)))()
        for i, it in enumerate(items):
            base, k = it.f[0], it.f[1]
            pa, px, py = _gemv_args(f"batched item {i}", base, k, it.m, it.n, it.lda, it.A, it.x, it.y,
                                    native_dtype(base), base // 8)
            arr[i] = fb_gemv_desc(fmt(it.f), it.m, it.n, 0, it.lda, pa, px, py)
        plan = _P()
        _check(load().fb_gemv_batched_plan(arr, len(items), ctypes.byref(plan)))
        self._plan = plan

    def tune(self, reps: int = 10, stream=None) -> None:
        _check(load().fb_gemv_batched_tune(self._plan, reps, _stream(stream)))

    def launch(self, stream=None) -> None:
        _check(load().fb_gemv_batched_launch(self._plan, _stream(stream)))

    def loop(self, stream=None) -> None:
        _check(load().fb_gemv_batched_loop(self._plan, _stream(stream)))

    def loop_graph(self, stream=None) -> None:
        _check(load().fb_gemv_batched_loop_graph(self._plan, _stream(stream)))

    @property
    def nbytes(self) -> int:
        return load().fb_plan_bytes(self._plan)

    def config(self, i: int) -> int:
        return load().fb_plan_config(self._plan, i)

    def close(self) -> None:
        if self._plan:
            load().fb_plan_destroy(self._plan)
            self._plan = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- BLAS 3
GEMM_ALL_PRODUCTS = 1
GEMM_FOUR_PRODUCTS = 1    # the {32,3} name of GEMM_ALL_PRODUCTS
GEMM_FP64 = 2


def gemm(fa, fb, fc, M: int, N: int, K: int, A: torch.Tensor, B: torch.Tensor, C: torch.Tensor | None = None,
         lda: int | None = None, ldb: int | None = None, ldc: int | None = None, flags: int = 0, stream=None):
    lda = K if lda is None else lda
    ldb = N if ldb is None else ldb
    ldc = N if ldc is None else ldc
    if C is None:
        if fc[1] * 8 == fc[0]:
            C = torch.empty(M * ldc, dtype=native_dtype(fc[0]), device=A.device)
        else:
            C = torch.empty(M * ldc * fc[1], dtype=torch.uint8, device=A.device)
    if (M > 0 and K > 0 and lda < K) or (K > 0 and N > 0 and ldb < N) or (M > 0 and N > 0 and ldc < N):
        raise ValueError(f"gemm: leading dimensions ({lda}, {ldb}, {ldc}) below the row lengths ({K}, {N}, {N})")
    pa = _arg(A, "gemm: A", _mat_bytes(M, K, lda, fa[1]))
    pb = _arg(B, "gemm: B", _mat_bytes(K, N, ldb, fb[1]), None, A)
    pc = _arg(C, "gemm: C", _mat_bytes(M, N, ldc, fc[1]), _out_dtype(fc[0], fc[1]), A)
    _check(load().fb_gemm_ex(fmt(fa), fmt(fb), fmt(fc), M, N, K, pa, lda, pb, ldb, pc, ldc, flags,
                             _stream(stream)))
    return C
