"""CPU oracle for the multibyte ("flyte") floating-point scheme -- TEST INFRASTRUCTURE.

This package is the plain, slow reference that the HIP library is checked
against.  Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import it; the library itself never does.  The
arithmetic lives in ``flyte_oracle.c`` (plain C, compiled with gcc); this module
only builds that file and marshals numpy arrays into it.

Functions follow the paper (Anderson & Gregg, PACT 2016):
  unpack        Section 3.2 and Section 4.1 (shift up, zero-fill)
  pack          Sections 5.2 and 5.3 (round to nearest even on the G/R/S/P bits,
                carry into the exponent, NaN kept NaN)
  axpy          Section 3.1 (compute in the base type) with FP_CONTRACT on (Section 4.4)
  dot/gemv/gemm naive: sequential fma in the base type (the AT_LEAST accumulator,
                Section 4.4); exact: Kulisch long accumulator, rounded once.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "flyte_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_lock = threading.Lock()
_libs: dict[int, ctypes.CDLL] = {}

FORMATS = [(32, 2), (32, 3), (32, 4)] + [(64, k) for k in range(2, 9)]


def lib_path(mutation: int = 0) -> str:
    name = "libflyte_oracle.so" if mutation == 0 else f"libflyte_oracle_mut{mutation}.so"
    return os.path.join(_BUILD, name)


def build(mutation: int = 0, force: bool = False) -> str:
    """Compiles the oracle with gcc (``-ffp-contract=off``: only explicit fma)."""
    out = lib_path(mutation)
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(_SRC):
        return out
    os.makedirs(_BUILD, exist_ok=True)
    tmp = out + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", f"-DFBO_MUTATION={mutation}", _SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def _declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    c_int, c_u64, c_sz, c_i64, c_dbl, c_p = (ctypes.c_int, ctypes.c_uint64, ctypes.c_size_t,
                                              ctypes.c_int64, ctypes.c_double, ctypes.c_void_p)
    sig = {
        "fbo_format_valid": (c_int, [c_int, c_int]),
        "fbo_mant_bits": (c_int, [c_int, c_int]),
        "fbo_unpack_bits": (c_u64, [c_int, c_int, c_u64]),
        "fbo_pack_bits": (c_u64, [c_int, c_int, c_u64]),
        "fbo_unpack": (None, [c_int, c_int, c_p, c_p, c_sz]),
        "fbo_pack": (None, [c_int, c_int, c_p, c_p, c_sz]),
        "fbo_axpy": (None, [c_int, c_int, c_sz, c_dbl, c_p, c_p]),
        "fbo_dot_naive": (c_dbl, [c_int, c_int, c_sz, c_p, c_p]),
        "fbo_dot_exact": (c_dbl, [c_int, c_int, c_sz, c_p, c_p]),
        "fbo_gemv_naive": (None, [c_int, c_int, c_i64, c_i64, c_p, c_i64, c_p, c_p]),
        "fbo_gemv_exact": (None, [c_int, c_int, c_i64, c_i64, c_p, c_i64, c_p, c_p, c_p]),
        "fbo_gemm_entries": (None, [c_int, c_int, c_int, c_int, c_i64, c_p, c_i64, c_p, c_i64,
                                    c_i64, c_p, c_p, c_p, c_p]),
        "fbo_gemm_naive": (None, [c_int, c_int, c_int, c_int, c_i64, c_i64, c_i64, c_p, c_i64,
                                  c_p, c_i64, c_p, c_i64]),
        "fbo_mutation": (c_int, []),
        "fbo_pack_bits_mode": (c_u64, [c_int, c_int, c_u64, c_int]),
        "fbo_pack_mode": (None, [c_int, c_int, c_int, c_p, c_p, c_sz]),
        "fbo_axpy_mode": (None, [c_int, c_int, c_int, c_sz, c_dbl, c_p, c_p]),
        "fbo_scale": (None, [c_int, c_int, c_int, c_sz, c_dbl, c_p]),
        "fbo_nrm2_naive": (c_dbl, [c_int, c_int, c_sz, c_p]),
        "fbo_nrm2_exact": (c_dbl, [c_int, c_int, c_sz, c_p]),
        "fbo_gemv_t_naive": (None, [c_int, c_int, c_i64, c_i64, c_p, c_i64, c_p, c_p]),
        "fbo_gemv_t_exact": (None, [c_int, c_int, c_i64, c_i64, c_p, c_i64, c_p, c_p, c_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def load(mutation: int = 0) -> ctypes.CDLL:
    with _lock:
        if mutation not in _libs:
            path = lib_path(mutation)
            if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
                build(mutation)
            _libs[mutation] = _declare(ctypes.CDLL(path))
        return _libs[mutation]


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _native_dtype(base: int):
    return np.float32 if base == 32 else np.float64


def _bits_dtype(base: int):
    return np.uint32 if base == 32 else np.uint64


def check_format(base: int, k: int) -> None:
    if not load().fbo_format_valid(base, k):
        raise ValueError(f"not a flyte format: base={base} k={k}")


class Oracle:
    """Numpy-facing wrappers around one build of the C oracle."""

    def __init__(self, mutation: int = 0):
        self.lib = load(mutation)
        self.mutation = mutation

    # -- single elements (integers in, integers out) -------------------
    def pack_bits(self, base: int, k: int, u: int) -> int:
        return int(self.lib.fbo_pack_bits(base, k, int(u)))

    def unpack_bits(self, base: int, k: int, q: int) -> int:
        return int(self.lib.fbo_unpack_bits(base, k, int(q)))

    def mant_bits(self, base: int, k: int) -> int:
        return int(self.lib.fbo_mant_bits(base, k))

    def pack_bits_mode(self, base: int, k: int, u: int, mode: int) -> int:
        return int(self.lib.fbo_pack_bits_mode(base, k, int(u), mode))

    # -- arrays ---------------------------------------------------------
    def pack(self, base: int, k: int, native: np.ndarray, mode: int = 0) -> np.ndarray:
        """native (float32/float64 or same-width uint bit patterns) -> uint8[n*k].

        mode: 0 round to nearest even, 1 toward zero, 2 to odd."""
        check_format(base, k)
        src = np.ascontiguousarray(native).view(_bits_dtype(base)).reshape(-1)
        out = np.empty(src.size * k, dtype=np.uint8)
        if mode == 0:
            self.lib.fbo_pack(base, k, _ptr(src), _ptr(out), src.size)
        else:
            self.lib.fbo_pack_mode(base, k, mode, _ptr(src), _ptr(out), src.size)
        return out

    def unpack(self, base: int, k: int, packed: np.ndarray, n: int | None = None) -> np.ndarray:
        """uint8[n*k] -> native array (float32/float64)."""
        check_format(base, k)
        src = np.ascontiguousarray(packed, dtype=np.uint8).reshape(-1)
        if n is None:
            n = src.size // k
        assert src.size >= n * k
        out = np.empty(n, dtype=_native_dtype(base))
        self.lib.fbo_unpack(base, k, _ptr(src), _ptr(out), n)
        return out

    def pack_u64(self, base: int, k: int, bits: np.ndarray) -> np.ndarray:
        """Element-wise pack on an array of bit patterns; returns the k-byte integers as uint64."""
        packed = self.pack(base, k, np.ascontiguousarray(bits).astype(_bits_dtype(base)))
        b = packed.reshape(-1, k).astype(np.uint64)
        q = np.zeros(b.shape[0], dtype=np.uint64)
        for j in range(k):
            q |= b[:, j] << np.uint64(8 * j)
        return q

    def axpy(self, base: int, k: int, alpha: float, x: np.ndarray, y: np.ndarray, mode: int = 0) -> np.ndarray:
        """Returns a new packed y <- pack(fma(alpha, x, y))."""
        x = np.ascontiguousarray(x, dtype=np.uint8).reshape(-1)
        yy = np.array(y, dtype=np.uint8, copy=True).reshape(-1)
        n = yy.size // k
        if mode == 0:
            self.lib.fbo_axpy(base, k, n, float(alpha), _ptr(x), _ptr(yy))
        else:
            self.lib.fbo_axpy_mode(base, k, mode, n, float(alpha), _ptr(x), _ptr(yy))
        return yy

    def scale(self, base: int, k: int, alpha: float, x: np.ndarray, mode: int = 0) -> np.ndarray:
        """Returns a new packed x <- pack(alpha * x)."""
        xx = np.array(x, dtype=np.uint8, copy=True).reshape(-1)
        self.lib.fbo_scale(base, k, mode, xx.size // k, float(alpha), _ptr(xx))
        return xx

    def nrm2_naive(self, base: int, k: int, x: np.ndarray) -> float:
        x = np.ascontiguousarray(x, dtype=np.uint8).reshape(-1)
        return float(self.lib.fbo_nrm2_naive(base, k, x.size // k, _ptr(x)))

    def nrm2_exact(self, base: int, k: int, x: np.ndarray) -> float:
        x = np.ascontiguousarray(x, dtype=np.uint8).reshape(-1)
        return float(self.lib.fbo_nrm2_exact(base, k, x.size // k, _ptr(x)))

    def dot_naive(self, base: int, k: int, x: np.ndarray, y: np.ndarray) -> float:
        x = np.ascontiguousarray(x, dtype=np.uint8).reshape(-1)
        y = np.ascontiguousarray(y, dtype=np.uint8).reshape(-1)
        return float(self.lib.fbo_dot_naive(base, k, x.size // k, _ptr(x), _ptr(y)))

    def dot_exact(self, base: int, k: int, x: np.ndarray, y: np.ndarray) -> float:
        x = np.ascontiguousarray(x, dtype=np.uint8).reshape(-1)
        y = np.ascontiguousarray(y, dtype=np.uint8).reshape(-1)
        return float(self.lib.fbo_dot_exact(base, k, x.size // k, _ptr(x), _ptr(y)))

    def gemv_naive(self, base: int, k: int, m: int, n: int, A: np.ndarray, lda: int,
                   x: np.ndarray) -> np.ndarray:
        A = np.ascontiguousarray(A, dtype=np.uint8).reshape(-1)
        x = np.ascontiguousarray(x, dtype=_native_dtype(base))
        y = np.empty(m, dtype=_native_dtype(base))
        self.lib.fbo_gemv_naive(base, k, m, n, _ptr(A), lda, _ptr(x), _ptr(y))
        return y

    def gemv_exact(self, base: int, k: int, m: int, n: int, A: np.ndarray, lda: int,
                   x: np.ndarray, rows: np.ndarray | None = None):
        """Exact y (rounded once to the base type, returned as float64) and sum |A||x| per row.

        ``rows`` restricts the work to a subset of rows (sampled checks)."""
        A = np.ascontiguousarray(A, dtype=np.uint8).reshape(-1)
        x = np.ascontiguousarray(x, dtype=_native_dtype(base))
        if rows is None:
            y = np.empty(m, dtype=np.float64)
            ab = np.empty(m, dtype=np.float64)
            self.lib.fbo_gemv_exact(base, k, m, n, _ptr(A), lda, _ptr(x), _ptr(y), _ptr(ab))
            return y, ab
        rows = np.asarray(rows, dtype=np.int64)
        y = np.empty(rows.size, dtype=np.float64)
        ab = np.empty(rows.size, dtype=np.float64)
        rowbytes = lda * k
        for t, r in enumerate(rows):
            seg = np.ascontiguousarray(A[int(r) * rowbytes:int(r) * rowbytes + n * k])
            yy = np.empty(1, dtype=np.float64)
            aa = np.empty(1, dtype=np.float64)
            self.lib.fbo_gemv_exact(base, k, 1, n, _ptr(seg), lda, _ptr(x), _ptr(yy), _ptr(aa))
            y[t], ab[t] = yy[0], aa[0]
        return y, ab

    def gemv_t_naive(self, base: int, k: int, m: int, n: int, A: np.ndarray, lda: int,
                     x: np.ndarray) -> np.ndarray:
        """y = A^T x, sequential fma over rows per column."""
        A = np.ascontiguousarray(A, dtype=np.uint8).reshape(-1)
        x = np.ascontiguousarray(x, dtype=_native_dtype(base))
        y = np.empty(n, dtype=_native_dtype(base))
        self.lib.fbo_gemv_t_naive(base, k, m, n, _ptr(A), lda, _ptr(x), _ptr(y))
        return y

    def gemv_t_exact(self, base: int, k: int, m: int, n: int, A: np.ndarray, lda: int, x: np.ndarray):
        """Exact y = A^T x (rounded once to the base type, as float64) and sum_i |A_ij x_i|."""
        A = np.ascontiguousarray(A, dtype=np.uint8).reshape(-1)
        x = np.ascontiguousarray(x, dtype=_native_dtype(base))
        y = np.empty(n, dtype=np.float64)
        ab = np.empty(n, dtype=np.float64)
        self.lib.fbo_gemv_t_exact(base, k, m, n, _ptr(A), lda, _ptr(x), _ptr(y), _ptr(ab))
        return y, ab

    def gemm_entries(self, fa, fb, K: int, A: np.ndarray, lda: int, B: np.ndarray, ldb: int,
                     ii: np.ndarray, jj: np.ndarray):
        """Exact C[i,j] (rounded once to binary64) and (|A||B|)[i,j] for the listed entries."""
        A = np.ascontiguousarray(A, dtype=np.uint8).reshape(-1)
        B = np.ascontiguousarray(B, dtype=np.uint8).reshape(-1)
        ii = np.ascontiguousarray(ii, dtype=np.int64)
        jj = np.ascontiguousarray(jj, dtype=np.int64)
        c = np.empty(ii.size, dtype=np.float64)
        ab = np.empty(ii.size, dtype=np.float64)
        self.lib.fbo_gemm_entries(fa[0], fa[1], fb[0], fb[1], K, _ptr(A), lda, _ptr(B), ldb,
                                  ii.size, _ptr(ii), _ptr(jj), _ptr(c), _ptr(ab))
        return c, ab

    def gemm_naive(self, fa, fb, M: int, N: int, K: int, A: np.ndarray, lda: int,
                   B: np.ndarray, ldb: int) -> np.ndarray:
        A = np.ascontiguousarray(A, dtype=np.uint8).reshape(-1)
        B = np.ascontiguousarray(B, dtype=np.uint8).reshape(-1)
        C = np.empty((M, N), dtype=np.float64)
        self.lib.fbo_gemm_naive(fa[0], fa[1], fb[0], fb[1], M, N, K, _ptr(A), lda, _ptr(B), ldb,
                                _ptr(C), N)
        return C


_default: Oracle | None = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle(0)
    return _default
