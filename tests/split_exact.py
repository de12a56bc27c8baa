"""Inputs on which every product of the split {32,3} GEMM operands, and every
partial sum of those products, is exact in binary32.

A {32,3} element keeps 15 mantissa bits.  The split products (the 3- and
4-product GEMMs) take hi = the element's top two bytes (a bfloat16: sign,
exponent, 7 mantissa bits) and lo = x - hi.  Elements here are

    a = s * 2^r * (h/4 + l * 2^-8),   h in {4, 5, 6, 7}, l in {0, 1}, s = +-1,

with r a per-row scale for A and a per-column scale for B, so hi = s 2^r h/4
and lo = s 2^r l 2^-8 (a non-zero lo for about half the elements).  In entry
(i, j) every product hi*hi, hi*lo, lo*hi and lo*lo is a multiple of
2^(r_i + c_j - 16) of magnitude below 2^(r_i + c_j + 2), and with K <= 64
every partial sum, in any order, is such a multiple below 2^(r_i + c_j + 8):
24 bits, exact in binary32.  So the four-product GEMM must return the exact
product bit for bit, and the three-product GEMM the exact product minus
sum_k lo(a_ik) lo(b_kj), also bit for bit; dropping any one product changes
some entry.
"""
from __future__ import annotations

import numpy as np

KMAX = 64


def values(rows: int, cols: int, seed: int, scale_axis: int) -> np.ndarray:
    """rows x cols float32 values of the form above; scale_axis 1 scales rows (A), 0 columns (B)."""
    g = np.random.default_rng(seed)
    h = g.integers(4, 8, (rows, cols)).astype(np.float64) / 4.0
    lo = g.integers(0, 2, (rows, cols)).astype(np.float64) * 2.0 ** -8
    s = g.choice([-1.0, 1.0], (rows, cols))
    if scale_axis == 1:
        r = g.integers(-3, 4, (rows, 1)).astype(np.float64)
    else:
        r = g.integers(-3, 4, (1, cols)).astype(np.float64)
    v = s * np.exp2(r) * (h + lo)
    out = v.astype(np.float32)
    assert np.array_equal(out.astype(np.float64), v)
    return out


def split(v: np.ndarray):
    """hi = the top two bytes of the binary32 pattern, lo = v - hi (both exact here)."""
    bits = np.ascontiguousarray(v, dtype=np.float32).view(np.uint32)
    hi = (bits & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
    return hi, v.astype(np.float64) - hi
