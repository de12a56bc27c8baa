"""Pins of the oracle's BLAS references (C3) against exact rational arithmetic.

* axpy (every rounding mode): fma(alpha, x, y) computed exactly with
  fractions, rounded once to the base type, then rounded to the flyte format
  with the independent rational rounding of ``valueround``; bit-exact.
* exact dot / gemv / gemm entries: the sum of products computed exactly with
  fractions and rounded once (binary64: Python's correctly rounded
  int/int division in ``float(Fraction)``; binary32: the rational rounder).
* naive dot / gemv: a case whose sequential-fma result is known in closed form,
  and integer data on which every order is exact (numpy matmul agrees).
* special values: NaN and infinities in dot products.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import oracle
import valueround as vr
from paper_1601_07789_amd import workloads

FORMATS = oracle.FORMATS


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


def bits_dtype(base):
    return np.uint32 if base == 32 else np.uint64


def native_dtype(base):
    return np.float32 if base == 32 else np.float64


def wide_values(n, seed, base):
    """Finite values over a wide exponent range, with some subnormals and zeros."""
    g = np.random.default_rng(seed)
    if base == 32:
        v = (g.standard_normal(n) * np.exp2(g.uniform(-30, 30, n))).astype(np.float32)
        sub = g.integers(1, 1 << 23, n // 10).astype(np.uint32).view(np.float32)
    else:
        v = g.standard_normal(n) * np.exp2(g.uniform(-200, 200, n))
        sub = g.integers(1, 1 << 52, n // 10, dtype=np.uint64).view(np.float64)
    v[: n // 10] = sub
    v[n // 10: n // 10 + 3] = 0.0
    g.shuffle(v)
    return v


def frac_of_packed(orc, base, k, packed):
    vals = orc.unpack(base, k, packed)
    return [vr.decode(base, int(u)) for u in vals.view(bits_dtype(base))]


# ---------------------------------------------------------------- axpy
@pytest.mark.parametrize("base,k", FORMATS)
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_axpy_vs_rational(orc, base, k, mode):
    """Every rounding mode: the exact fma in fractions, rounded once to the
    base type, then cut to k bytes by the independent rational rounder in that
    mode (nearest even, Section 5.2; toward zero, Section 5.1; to odd,
    Section 7).  Mode 0 goes through fbo_axpy, the others through
    fbo_axpy_mode."""
    n = 600
    x = orc.pack(base, k, wide_values(n, 11 + k, base))
    y = orc.pack(base, k, wide_values(n, 12 + k, base))
    alpha = float.fromhex("0x1.5555555555555p-2")   # RN(1/3) in binary64
    got = orc.axpy(base, k, alpha, x, y, mode)
    a_native = np.float32(alpha) if base == 32 else alpha
    a = Fraction(float(a_native))
    xs, ys = frac_of_packed(orc, base, k, x), frac_of_packed(orc, base, k, y)
    gq = orc.pack_u64(base, k, orc.unpack(base, k, got).view(bits_dtype(base)))
    E, m, bias, emin, emax = vr.params(base, k)
    for i in range(n):
        exact = a * xs[i] + ys[i]
        r = vr.round_to_base(exact, base)          # the single fma rounding
        neg = (r == vr.NINF) or (r not in (vr.INF, vr.NINF) and r < 0)
        if r not in (vr.INF, vr.NINF) and r == 0:
            # sign of an exact zero sum under round-to-nearest: + unless both terms are -0
            neg = False
        if r in (vr.INF, vr.NINF):
            rk = r
        elif mode == 0:
            rk = vr.round_rne(r, m + 1, emin, emax)
        else:
            rk = vr.round_directed(r, m + 1, emin, mode)
        want = vr.encode(base, k, rk, neg)
        assert int(gq[i]) == want, (i, base, k, mode)


def test_axpy_specials(orc):
    base, k = 64, 5
    xv = np.array([np.nan, np.inf, 1.0, -np.inf, 0.0], dtype=np.float64)
    yv = np.array([1.0, 1.0, np.nan, np.inf, -0.0], dtype=np.float64)
    got = orc.unpack(base, k, orc.axpy(base, k, 2.0, orc.pack(base, k, xv), orc.pack(base, k, yv)))
    assert np.isnan(got[0]) and got[1] == np.inf and np.isnan(got[2]) and np.isnan(got[3])
    assert got[4] == 0.0


# ---------------------------------------------------------------- dot
def exact_dot_frac(xs, ys):
    return sum((a * b for a, b in zip(xs, ys)), Fraction(0))


@pytest.mark.parametrize("base,k", FORMATS)
def test_dot_exact_vs_rational(orc, base, k):
    for seed in range(3):
        n = 257 + 100 * seed
        x = orc.pack(base, k, wide_values(n, 100 + seed, base))
        y = orc.pack(base, k, wide_values(n, 200 + seed, base))
        exact = exact_dot_frac(frac_of_packed(orc, base, k, x), frac_of_packed(orc, base, k, y))
        want = vr.to_float(vr.round_to_base(exact, base))
        got = orc.dot_exact(base, k, x, y)
        assert got == want or (got == 0 and want == 0), (base, k, seed, got, want)


def test_dot_exact_cancellation_and_tiny(orc):
    """Massive cancellation and a sub-ulp residue: only an exact sum gets these right."""
    big = 2.0 ** 900
    xv = np.array([big, 1.0, -big, 2.0 ** -1074, 3.0], dtype=np.float64)
    yv = np.array([big, 2.0 ** -1070, big, 1.0, 2.0 ** -1074], dtype=np.float64)
    # terms: 2^1800 + 2^-1070 - 2^1800 + 2^-1074 + 3*2^-1074 = 2^-1070 + 2^-1072
    # but 2^1800 overflows binary64 -> the exact accumulator must still cancel it
    x = orc.pack(64, 8, xv)
    y = orc.pack(64, 8, yv)
    assert orc.dot_exact(64, 8, x, y) == 2.0 ** -1070 + 2.0 ** -1072
    # a tie between two subnormals: exact value 2^-1075 rounds to even (0)
    x = orc.pack(64, 8, np.array([2.0 ** -1000], dtype=np.float64))
    y = orc.pack(64, 8, np.array([2.0 ** -75], dtype=np.float64))
    assert orc.dot_exact(64, 8, x, y) == 0.0
    y = orc.pack(64, 8, np.array([3.0 * 2.0 ** -76], dtype=np.float64))
    assert orc.dot_exact(64, 8, x, y) == 2.0 ** -1074   # 1.5 * 2^-1075 rounds up


def test_dot_specials(orc):
    f = lambda v: orc.pack(64, 8, np.array(v, dtype=np.float64))
    assert np.isnan(orc.dot_exact(64, 8, f([1.0, np.nan]), f([1.0, 1.0])))
    assert orc.dot_exact(64, 8, f([np.inf, 1.0]), f([2.0, 1.0])) == np.inf
    assert orc.dot_exact(64, 8, f([np.inf, 1.0]), f([-2.0, 1.0])) == -np.inf
    assert np.isnan(orc.dot_exact(64, 8, f([np.inf, np.inf]), f([1.0, -1.0])))
    assert np.isnan(orc.dot_exact(64, 8, f([np.inf]), f([0.0])))
    # finite overflow of the exact value rounds to infinity
    big = np.finfo(np.float64).max
    assert orc.dot_exact(64, 8, f([big, big]), f([1.0, 1.0])) == np.inf
    assert np.isnan(orc.dot_naive(64, 8, f([1.0, np.nan]), f([1.0, 1.0])))


def test_dot_naive_is_sequential_fma(orc):
    """Closed form: the sequential fma chain loses the small middle term."""
    x = orc.pack(64, 8, np.array([1.0, 2.0 ** -60, -1.0]))
    y = orc.pack(64, 8, np.array([1.0, 1.0, 1.0]))
    assert orc.dot_naive(64, 8, x, y) == 0.0
    assert orc.dot_exact(64, 8, x, y) == 2.0 ** -60
    # fma contraction: x*y is not rounded before the add
    a = 1.0 + 2.0 ** -30
    x = orc.pack(64, 8, np.array([a, -1.0]))
    y = orc.pack(64, 8, np.array([a, 1.0 + 2.0 ** -29]))
    # first step: fma(a, a, 0) = RN(1 + 2^-29 + 2^-60) = 1 + 2^-29; then fma(-1, 1+2^-29, that) = 0
    assert orc.dot_naive(64, 8, x, y) == 0.0
    assert orc.dot_exact(64, 8, x, y) == 2.0 ** -60
    # the other order shows the contraction: fma(-1, 1+2^-29, 0) = -(1+2^-29) exactly, then
    # fma(a, a, -(1+2^-29)) keeps the 2^-60 of the unrounded product; a separate multiply
    # and add would round a*a to 1+2^-29 first and return 0
    x = orc.pack(64, 8, np.array([-1.0, a]))
    y = orc.pack(64, 8, np.array([1.0 + 2.0 ** -29, a]))
    assert orc.dot_naive(64, 8, x, y) == 2.0 ** -60


@pytest.mark.parametrize("base,k", FORMATS)
def test_dot_integer_data_exact_in_any_order(orc, base, k):
    g = np.random.default_rng(5)
    p = min(8, vr.params(base, k)[1] + 1)   # integers with at most p bits are exact in the format
    xv = g.integers(-(1 << (p - 1)), 1 << (p - 1), 1000).astype(native_dtype(base))
    yv = g.integers(-(1 << (p - 1)), 1 << (p - 1), 1000).astype(native_dtype(base))
    x, y = orc.pack(base, k, xv), orc.pack(base, k, yv)
    want = float(np.dot(xv.astype(np.int64), yv.astype(np.int64)))
    assert orc.dot_naive(base, k, x, y) == want
    assert orc.dot_exact(base, k, x, y) == want


# ---------------------------------------------------------------- gemv
@pytest.mark.parametrize("base,k", [(32, 2), (32, 3), (64, 3), (64, 5), (64, 8)])
def test_gemv_exact_vs_rational(orc, base, k):
    m, n, lda = 7, 37, 40
    A = orc.pack(base, k, wide_values(m * lda, 300 + k, base))
    x = wide_values(n, 400 + k, base)
    y, ab = orc.gemv_exact(base, k, m, n, A, lda, x)
    rowbytes = lda * k
    xf = [vr.decode(base, int(u)) for u in x.view(bits_dtype(base))]
    for r in range(m):
        av = frac_of_packed(orc, base, k, A[r * rowbytes:r * rowbytes + n * k])
        exact = exact_dot_frac(av, xf)
        assert y[r] == vr.to_float(vr.round_to_base(exact, base))
        assert ab[r] == float(sum((abs(a * b) for a, b in zip(av, xf)), Fraction(0)))
    rows = np.array([6, 0, 3])
    ys, _ = orc.gemv_exact(base, k, m, n, A, lda, x, rows=rows)
    assert np.array_equal(ys, y[rows])


@pytest.mark.parametrize("base,k", [(32, 3), (64, 6)])
def test_gemv_naive_integer_data(orc, base, k):
    g = np.random.default_rng(9)
    m, n, lda = 33, 70, 72
    Av = g.integers(-100, 100, (m, lda)).astype(native_dtype(base))
    xv = g.integers(-100, 100, n).astype(native_dtype(base))
    A = orc.pack(base, k, Av.reshape(-1))
    y = orc.gemv_naive(base, k, m, n, A, lda, xv)
    assert np.array_equal(y, (Av[:, :n].astype(np.int64) @ xv.astype(np.int64)).astype(native_dtype(base)))


@pytest.mark.parametrize("base,k", [(32, 3), (64, 5), (64, 8)])
def test_gemv_t_exact_vs_rational(orc, base, k):
    m, n, lda = 41, 9, 12
    A = orc.pack(base, k, wide_values(m * lda, 500 + k, base))
    x = wide_values(m, 600 + k, base)
    y, ab = orc.gemv_t_exact(base, k, m, n, A, lda, x)
    rowbytes = lda * k
    xf = [vr.decode(base, int(u)) for u in x.view(bits_dtype(base))]
    Af = [frac_of_packed(orc, base, k, A[r * rowbytes:r * rowbytes + n * k]) for r in range(m)]
    for c in range(n):
        terms = [Af[r][c] * xf[r] for r in range(m)]
        assert y[c] == vr.to_float(vr.round_to_base(sum(terms, Fraction(0)), base))
        assert ab[c] == float(sum((abs(t) for t in terms), Fraction(0)))


def test_gemv_t_naive_integer_data_and_order(orc):
    g = np.random.default_rng(12)
    m, n = 37, 21
    Av = g.integers(-100, 100, (m, n)).astype(np.float64)
    xv = g.integers(-100, 100, m).astype(np.float64)
    A = orc.pack(64, 6, Av.reshape(-1))
    assert np.array_equal(orc.gemv_t_naive(64, 6, m, n, A, n, xv), Av.T @ xv)
    # sequential over rows: the small middle term is lost, as in the dot closed form
    A = orc.pack(64, 8, np.array([[1.0], [2.0 ** -60], [-1.0]]).reshape(-1))
    assert orc.gemv_t_naive(64, 8, 3, 1, A, 1, np.ones(3))[0] == 0.0


# ---------------------------------------------------------------- gemm
def test_gemm_entries_vs_rational(orc):
    g = np.random.default_rng(3)
    M, N, K = 5, 6, 33
    lda, ldb = K + 3, N + 2      # padded rows: the leading dimensions must be honoured
    for fa in [(32, 2), (32, 3), (64, 5), (64, 6)]:
        base, k = fa
        Av = (g.standard_normal((M, lda)) * np.exp2(g.uniform(-20, 20, (M, lda)))).astype(native_dtype(base))
        Bv = (g.standard_normal((K, ldb)) * np.exp2(g.uniform(-20, 20, (K, ldb)))).astype(native_dtype(base))
        A, B = orc.pack(base, k, Av.reshape(-1)), orc.pack(base, k, Bv.reshape(-1))
        ii, jj = np.array([0, 4, 2]), np.array([5, 0, 3])
        c, cab = orc.gemm_entries(fa, fa, K, A, lda, B, ldb, ii, jj)
        Au = orc.unpack(base, k, A).reshape(M, lda)
        Bu = orc.unpack(base, k, B).reshape(K, ldb)
        for t in range(3):
            i, j = ii[t], jj[t]
            terms = [Fraction(float(Au[i, p])) * Fraction(float(Bu[p, j])) for p in range(K)]
            assert c[t] == float(sum(terms, Fraction(0)))
            assert cab[t] == float(sum((abs(z) for z in terms), Fraction(0)))


def test_gemm_naive_integer_data(orc):
    g = np.random.default_rng(4)
    M, N, K = 9, 11, 13
    Av = g.integers(-50, 50, (M, K)).astype(np.float64)
    Bv = g.integers(-50, 50, (K, N)).astype(np.float64)
    A, B = orc.pack(64, 5, Av.reshape(-1)), orc.pack(64, 5, Bv.reshape(-1))
    C = orc.gemm_naive((64, 5), (64, 5), M, N, K, A, K, B, N)
    assert np.array_equal(C, Av @ Bv)


# ---------------------------------------------------------------- workloads sanity (generator only)
def test_mixed_population_composition():
    bits = workloads.mixed_binary64(1 << 14, workloads.SEED_BASE)
    v = bits.view(np.float64)
    assert np.isnan(v).sum() > 0 and np.isinf(v).sum() > 0
    assert (bits == np.uint64(0x7FF0000000000001)).any()
    frac_special = 1 - np.isfinite(v).mean()
    assert 0.02 < frac_special < 0.05        # infinities + NaNs are 3 of the 9 special kinds


# ---------------------------------------------------------------- planted mistakes in the BLAS references
BLAS_MUTATIONS = {
    7: ("exact accumulator ignores the sign of products",
        [lambda o: test_dot_exact_vs_rational(o, 64, 5), lambda o: test_dot_exact_cancellation_and_tiny(o)]),
    8: ("transposed GEMV multiplies by the wrong x index",
        [lambda o: test_gemv_t_exact_vs_rational(o, 64, 3)]),
    9: ("axpy computes alpha*y + x", [lambda o: test_axpy_vs_rational(o, 32, 3, 0),
                                      lambda o: test_axpy_vs_rational(o, 64, 5, 2)]),
    10: ("naive dot rounds each product before adding", [lambda o: test_dot_naive_is_sequential_fma(o)]),
    11: ("axpy ignores its rounding mode", [lambda o: test_axpy_vs_rational(o, 64, 5, 1),
                                           lambda o: test_axpy_vs_rational(o, 32, 3, 2)]),
}


@pytest.mark.parametrize("mut", sorted(BLAS_MUTATIONS))
def test_planted_blas_mutation_is_caught(mut):
    oracle.build(mut)
    o = oracle.Oracle(mut)
    assert o.lib.fbo_mutation() == mut
    failed = 0
    for pin in BLAS_MUTATIONS[mut][1]:
        try:
            pin(o)
        except AssertionError:
            failed += 1
    assert failed > 0, BLAS_MUTATIONS[mut][0]
