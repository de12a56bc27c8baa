"""CPU pins of the split-product GEMM parity tests (no GPU).

The GPU tests of the 3- and 4-product GEMMs ({32,3} operands split into
bfloat16 hi and lo) compare bit for bit on inputs built so that every product
of split operands and every partial sum is exact in binary32 (``split_exact``).
This file shows, with a numpy model of the split products, that those
comparisons discriminate:

* the construction is exact: the model in binary32, summed in three different
  orders, equals the oracle's exact product (four products) and the exact
  product minus the lo*lo sum (three products);
* every variant that drops one of the products it should form, or adds lo*lo
  to the three products, misses the expected values in some entry;
* the split keeps NaN: a {32,3} NaN whose payload lies only in its low byte
  (pattern 7F8001) would have a bfloat16 hi with a zero mantissa, an
  infinity, unless the split sets its quiet bit.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import oracle
import split_exact

PRODUCTS = ("hh", "hl", "lh", "ll")


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


def model(Ah, Al, Bh, Bl, products, order):
    """Sum over k of the chosen products, accumulated in binary32 in the given k order."""
    terms = {"hh": (Ah, Bh), "hl": (Ah, Bl), "lh": (Al, Bh), "ll": (Al, Bl)}
    M, K = Ah.shape
    N = Bh.shape[1]
    acc = np.zeros((M, N), dtype=np.float32)
    for kk in order:
        for p in products:
            a, b = terms[p]
            prod = np.outer(a[:, kk], b[kk, :])          # exact in binary64
            assert np.array_equal(prod.astype(np.float32).astype(np.float64), prod)
            acc = (acc + prod.astype(np.float32)).astype(np.float32)
    return acc.astype(np.float64)


def construction(orc, M=32, N=48, K=64, seed=5):
    Av = split_exact.values(M, K, seed, 1)
    Bv = split_exact.values(K, N, seed + 1, 0)
    A, B = orc.pack(32, 3, Av.reshape(-1)), orc.pack(32, 3, Bv.reshape(-1))
    # the values are {32,3} elements: packing keeps them
    assert np.array_equal(orc.unpack(32, 3, A).reshape(M, K), Av)
    assert np.array_equal(orc.unpack(32, 3, B).reshape(K, N), Bv)
    ii, jj = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
    exact, _ = orc.gemm_entries((32, 3), (32, 3), K, A, K, B, N, ii.reshape(-1), jj.reshape(-1))
    Ah, Al = split_exact.split(Av)
    Bh, Bl = split_exact.split(Bv)
    return Av, Bv, exact.reshape(M, N), (Ah, Al, Bh, Bl)


def test_lo_is_nonzero_and_small(orc):
    Av, Bv, exact, (Ah, Al, Bh, Bl) = construction(orc)
    for v, lo in ((Av, Al), (Bv, Bl)):
        frac = np.mean(lo != 0)
        assert 0.3 < frac < 0.7
        assert np.all(np.abs(lo) <= np.abs(v) * 2.0 ** -8)


@pytest.mark.parametrize("order", ["forward", "reverse", "interleaved"])
def test_construction_is_exact(orc, order):
    Av, Bv, exact, parts = construction(orc)
    K = Av.shape[1]
    ks = {"forward": range(K), "reverse": range(K - 1, -1, -1),
          "interleaved": list(range(0, K, 2)) + list(range(1, K, 2))}[order]
    _, Al, _, Bl = parts
    assert np.array_equal(model(*parts, PRODUCTS, ks), exact)
    lolo = Al @ Bl
    assert np.array_equal(model(*parts, ("hh", "hl", "lh"), ks), exact - lolo)
    assert np.any(lolo != 0)


def test_every_dropped_product_is_caught(orc):
    Av, Bv, exact, parts = construction(orc)
    _, Al, _, Bl = parts
    K = Av.shape[1]
    want4, want3 = exact, exact - Al @ Bl
    for r in range(0, 4):
        for subset in itertools.combinations(PRODUCTS, r):
            got = model(*parts, subset, range(K))
            assert not np.array_equal(got, want4), subset
            if set(subset) != {"hh", "hl", "lh"}:
                assert not np.array_equal(got, want3), subset
    # the three-product expectation also rejects the four products
    assert not np.array_equal(model(*parts, PRODUCTS, range(K)), want3)


def split_bits(u: int):
    """hi and lo (bfloat16 patterns) of a binary32 pattern, with the NaN rule of the split."""
    hi = u >> 16
    if (u & 0x7FFFFFFF) > 0x7F800000:
        hi |= 0x40
    if (u & 0x7F800000) == 0x7F800000:
        return hi, 0
    x = np.array([u], dtype=np.uint32).view(np.float32)[0]
    h = np.array([u & 0xFFFF0000], dtype=np.uint32).view(np.float32)[0]
    return hi, int(np.array([x - h], dtype=np.float32).view(np.uint32)[0]) >> 16


def bf16(p: int) -> float:
    return float(np.array([p << 16], dtype=np.uint32).view(np.float32)[0])


def test_split_keeps_low_byte_nan(orc):
    u = 0x7F800100                      # {32,3} pattern 7F8001: a NaN with payload only in the low byte
    q = orc.pack(32, 3, np.array([u], dtype=np.uint32).view(np.float32))
    assert bytes(q) == bytes([0x01, 0x80, 0x7F])   # packing keeps it (the kept mantissa is non-zero)
    assert (u >> 16) == 0x7F80                      # without the rule hi would be +Inf
    hi, lo = split_bits(u)
    assert np.isnan(bf16(hi)) and lo == 0
    # against a finite non-zero partner the rule gives NaN, the plain top two bytes Inf
    assert np.isnan(bf16(hi) * 1.5)
    assert np.isinf(bf16(u >> 16) * 1.5)
    for u2 in (0x7FC00000, 0xFF800001, 0x7F800000, 0xFF800000):
        h2, l2 = split_bits(u2)
        assert np.isnan(bf16(h2)) == np.isnan(np.array([u2], dtype=np.uint32).view(np.float32)[0])
        assert l2 == 0
