"""Exact rational rounding, independent of the oracle (test helper).

Everything here works on values, with ``fractions.Fraction``: decode an IEEE
bit pattern to its exact rational value, round a rational to nearest-even on the
grid of a floating-point format with given precision and exponent range, and
encode a rational that lies on that grid back into sign/exponent/mantissa
fields.  It shares no code with the C oracle, and so gives independent pins for
its bit-level pack (Sections 5.2 and 5.3 of the paper) and for its exact
dot-product reference.
"""
from __future__ import annotations

from fractions import Fraction

INF = "inf"
NINF = "-inf"


def params(base: int, k: int):
    """(E, m, bias, emin, emax) of the flyte format {base, k} (Table 1 rule m = 8k-1-E)."""
    E = 8 if base == 32 else 11
    m = 8 * k - 1 - E
    bias = (1 << (E - 1)) - 1
    return E, m, bias, 1 - bias, bias


def decode(base: int, u: int):
    """Exact value of a binary32/binary64 bit pattern: Fraction, INF, NINF or 'nan'."""
    E = 8 if base == 32 else 11
    M = base - 1 - E
    bias = (1 << (E - 1)) - 1
    s = (u >> (base - 1)) & 1
    e = (u >> M) & ((1 << E) - 1)
    f = u & ((1 << M) - 1)
    if e == (1 << E) - 1:
        if f:
            return "nan"
        return NINF if s else INF
    if e == 0:
        v = Fraction(f, 1) * Fraction(2) ** (1 - bias - M)
    else:
        v = Fraction((1 << M) | f, 1) * Fraction(2) ** (e - bias - M)
    return -v if s else v


def floor_log2(a: Fraction) -> int:
    """floor(log2(a)) for a > 0, exactly."""
    n, d = a.numerator, a.denominator
    e = n.bit_length() - d.bit_length()
    # adjust so that 2^e <= a < 2^(e+1)
    if e >= 0:
        if n < (d << e):
            e -= 1
    else:
        if (n << -e) < d:
            e -= 1
    return e


def round_rne(v: Fraction, p: int, emin: int, emax: int):
    """Round v to nearest (ties to even) with precision p, normal range [emin, emax],
    gradual underflow.  Returns a Fraction (zero carries no sign; callers track it)
    or INF/NINF on overflow."""
    if v == 0:
        return Fraction(0)
    neg = v < 0
    a = -v if neg else v
    e = floor_log2(a)
    s = max(e, emin) - (p - 1)
    scale = Fraction(2) ** s
    q = a / scale
    n = q.numerator // q.denominator
    rem = q - n
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and n % 2 == 1):
        n += 1
    r = n * scale
    if r >= Fraction(2) ** (emax + 1):
        return NINF if neg else INF
    return -r if neg else r


def encode(base: int, k: int, v, negative: bool) -> int:
    """k-byte pattern of a value already on the format's grid (or INF/NINF)."""
    E, m, bias, emin, emax = params(base, k)
    sign = 1 if negative else 0
    top = sign << (8 * k - 1)
    if v == INF or v == NINF:
        return top | (((1 << E) - 1) << m)
    a = abs(v)
    if a == 0:
        return top
    e = floor_log2(a)
    if e < emin:
        mant = a / Fraction(2) ** (emin - m)
        assert mant.denominator == 1 and mant.numerator < (1 << m)
        return top | mant.numerator
    mant = a / Fraction(2) ** (e - m)
    assert mant.denominator == 1 and (1 << m) <= mant.numerator < (1 << (m + 1))
    return top | ((e + bias) << m) | (mant.numerator - (1 << m))


def expected_pack(base: int, k: int, u: int):
    """Expected k-byte pattern for a non-NaN input pattern u; None for NaN inputs."""
    val = decode(base, u)
    neg = bool((u >> (base - 1)) & 1)
    if val == "nan":
        return None
    E, m, bias, emin, emax = params(base, k)
    if val in (INF, NINF):
        return encode(base, k, val, neg)
    return encode(base, k, round_rne(val, m + 1, emin, emax), neg)


def round_directed(v: Fraction, p: int, emin: int, mode: int):
    """Round toward zero (mode 1) or to odd (mode 2) with precision p and minimum
    normal exponent emin (gradual underflow); never overflows."""
    if v == 0:
        return Fraction(0)
    neg = v < 0
    a = -v if neg else v
    e = floor_log2(a)
    s = max(e, emin) - (p - 1)
    scale = Fraction(2) ** s
    q = a / scale
    n = q.numerator // q.denominator
    if mode == 2 and n * scale != a and n % 2 == 0:
        n += 1
    r = n * scale
    return -r if neg else r


def expected_pack_mode(base: int, k: int, u: int, mode: int):
    """Expected k-byte pattern for a non-NaN input in rounding mode 0, 1 or 2."""
    if mode == 0:
        return expected_pack(base, k, u)
    val = decode(base, u)
    neg = bool((u >> (base - 1)) & 1)
    if val == "nan":
        return None
    E, m, bias, emin, emax = params(base, k)
    if val in (INF, NINF):
        return encode(base, k, val, neg)
    return encode(base, k, round_directed(val, m + 1, emin, mode), neg)


def round_to_base(v, base: int):
    """Round an exact rational to binary32/binary64 (nearest even); INF/NINF on overflow."""
    if base == 32:
        return round_rne(v, 24, -126, 127)
    return round_rne(v, 53, -1022, 1023)


def to_float(v) -> float:
    if v == INF:
        return float("inf")
    if v == NINF:
        return float("-inf")
    return float(v)   # exact: v is representable in binary64 here
