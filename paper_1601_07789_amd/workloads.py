"""Seeded synthetic workloads for the flyte kernels.

Pure numpy, no packing or rounding: these functions only draw native values
(binary32/binary64 bit patterns, matrices, batch descriptors) with the shapes
and distributions of the benchmark workloads.  Both the CPU oracle (in tests)
and the HIP library consume the same draws; each side packs them itself.

Seeds: ``SEED_BASE + config index`` (0 round-trip + dot, 1 streaming BLAS,
2 precision GEMM, 3 batched GEMV, 4 FP64 GEMM); the second vector of a pair
uses ``+100``.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 160107789

# Every flyte format: binary32 with 2..4 bytes, binary64 with 2..8 bytes.
FORMATS = [(32, 2), (32, 3), (32, 4)] + [(64, k) for k in range(2, 9)]

_F64_MAX = 0x7FEFFFFFFFFFFFFF


def rng(config: int, offset: int = 0) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + config + offset)


def mixed_binary64(n: int, seed: int) -> np.ndarray:
    """binary64 bit patterns (uint64): 90% N(0,1) * 2^U(-60,60), 10% special values.

    The specials are split evenly over: signed zeros; subnormals (random
    payloads, plus the largest and smallest); infinities; quiet NaNs (random
    payload, both signs); signalling NaNs (payload only in the low bytes, and
    the largest payload); the largest finite magnitudes; exact rounding ties
    for a random cut k in 2..7 with a random kept lowest bit (including the
    tie just below infinity); and near-ties one binary64 ulp either side.
    """
    g = np.random.default_rng(seed)
    vals = g.standard_normal(n) * np.exp2(g.uniform(-60.0, 60.0, n))
    bits = vals.view(np.uint64).copy()
    n_spec = n // 10
    idx = g.permutation(n)[:n_spec]
    kinds = np.arange(n_spec) % 9
    g.shuffle(kinds)
    sign = (g.integers(0, 2, n_spec, dtype=np.uint64) << np.uint64(63))
    mant52 = g.integers(1, 1 << 52, n_spec, dtype=np.uint64)
    out = np.empty(n_spec, dtype=np.uint64)
    for t in range(9):
        sel = kinds == t
        cnt = int(sel.sum())
        s = sign[sel]
        if t == 0:          # signed zeros
            v = s
        elif t == 1:        # subnormals
            v = s | mant52[sel]
            if cnt >= 2:
                v[0] = 0x000FFFFFFFFFFFFF
                v[1] = 0x0000000000000001
        elif t == 2:        # infinities
            v = s | np.uint64(0x7FF0000000000000)
        elif t == 3:        # quiet NaNs, random payload
            v = s | np.uint64(0x7FF8000000000000) | (mant52[sel] & np.uint64((1 << 51) - 1))
        elif t == 4:        # signalling NaNs, payload in the low bytes
            low = g.integers(1, 1 << 16, cnt, dtype=np.uint64)
            v = s | np.uint64(0x7FF0000000000000) | low
            if cnt >= 2:
                v[0] = 0x7FF0000000000001
                v[1] = 0x7FF7FFFFFFFFFFFF
        elif t == 5:        # largest finite magnitudes
            v = s | np.uint64(_F64_MAX)
        elif t in (6, 7, 8):  # exact ties and near-ties at a random cut
            kk = g.integers(2, 8, cnt)
            d = (64 - 8 * kk).astype(np.uint64)
            expo = g.integers(1, 2047, cnt, dtype=np.uint64)
            top = (s | (expo << np.uint64(52)) | mant52[sel]) >> d << d
            half = np.uint64(1) << (d - np.uint64(1))
            v = top | half
            if t == 7:
                v = v + np.uint64(1)
            elif t == 8:
                v = v - np.uint64(1)
            if t == 6 and cnt >= 1:
                v[0] = 0x7FEFFFFFFFFFFFFF >> 16 << 16 | (1 << 15)   # tie just below infinity, k=6
        out[sel] = v
    bits[idx] = out
    return bits


def mixed_binary32(n: int, seed: int) -> np.ndarray:
    """binary32 bit patterns (uint32): 90% N(0,1) * 2^U(-30,30), 10% special values
    (signed zeros, subnormals, infinities, quiet and signalling NaNs, largest
    finite magnitudes, and exact ties / near-ties for a random cut k in 2..3)."""
    g = np.random.default_rng(seed)
    vals = (g.standard_normal(n) * np.exp2(g.uniform(-30.0, 30.0, n))).astype(np.float32)
    bits = vals.view(np.uint32).copy()
    n_spec = n // 10
    idx = g.permutation(n)[:n_spec]
    kinds = np.arange(n_spec) % 9
    g.shuffle(kinds)
    sign = g.integers(0, 2, n_spec, dtype=np.uint32) << np.uint32(31)
    mant = g.integers(1, 1 << 23, n_spec, dtype=np.uint32)
    out = np.empty(n_spec, dtype=np.uint32)
    for t in range(9):
        sel = kinds == t
        cnt = int(sel.sum())
        s = sign[sel]
        if t == 0:
            v = s
        elif t == 1:
            v = s | mant[sel]
        elif t == 2:
            v = s | np.uint32(0x7F800000)
        elif t == 3:
            v = s | np.uint32(0x7FC00000) | (mant[sel] & np.uint32((1 << 22) - 1))
        elif t == 4:
            v = s | np.uint32(0x7F800000) | g.integers(1, 1 << 8, cnt, dtype=np.uint32)
        elif t == 5:
            v = s | np.uint32(0x7F7FFFFF)
        else:
            kk = g.integers(2, 4, cnt)
            d = (32 - 8 * kk).astype(np.uint32)
            expo = g.integers(1, 255, cnt, dtype=np.uint32)
            top = (s | (expo << np.uint32(23)) | mant[sel]) >> d << d
            v = top | (np.uint32(1) << (d - np.uint32(1)))
            if t == 7:
                v = v + np.uint32(1)
            elif t == 8:
                v = v - np.uint32(1)
        out[sel] = v
    bits[idx] = out
    return bits


def uniform(n: int, seed: int, dtype=np.float64, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n).astype(dtype)


def normal(shape, seed: int, dtype=np.float32) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)


def small_integers(n: int, seed: int, dtype=np.float64, lo: int = -8, hi: int = 8) -> np.ndarray:
    """Integers in [lo, hi] as floating point: exact in every format with at least
    four kept mantissa bits, and their products and sums stay exact in binary64."""
    return np.random.default_rng(seed).integers(lo, hi + 1, n).astype(dtype)


def group_elems(k: int) -> int:
    """Elements per dword-aligned group: 4 / gcd(4, k)."""
    from math import gcd
    return 4 // gcd(4, k)


def batched_descs(count: int, seed: int, lo: int = 64, hi: int = 4096,
                  formats=FORMATS):
    """Shapes and formats of a batch of independent GEMVs.

    m and n are drawn independently as round(exp(U(ln lo, ln hi))); the format is
    uniform over ``formats``; lda is n rounded up to a multiple of the format's
    dword group so that every row starts on a 4-byte boundary.
    Returns a list of dicts {base, k, m, n, lda}.
    """
    g = np.random.default_rng(seed)
    m = np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), count))).astype(np.int64)
    nn = np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), count))).astype(np.int64)
    fi = g.integers(0, len(formats), count)
    out = []
    for t in range(count):
        base, k = formats[int(fi[t])]
        G = group_elems(k)
        lda = int((nn[t] + G - 1) // G * G)
        out.append({"base": base, "k": k, "m": int(m[t]), "n": int(nn[t]), "lda": lda})
    return out
