"""Pins of the oracle's other rounding modes, scale and magnitude.

* toward zero and to odd: the independent value-domain checker, exhaustive on
  every binary32 input (k = 2 both modes, k = 3 to odd); exact rational
  rounding on structured sweeps for every format; a hand-built table;
* the Boldo-Melquiond property of rounding to odd, exhaustive on binary32:
  nearest-even into k bytes after rounding to odd into k+1 bytes equals
  nearest-even into k bytes directly;
* a planted mutation (round to odd that never sets the odd bit) is caught;
* scale (x <- alpha x, in place) against exact rational arithmetic, bit-exact;
* magnitude (Euclidean norm) exact reference against fractions and a
  correctly rounded square root; the naive reference on a closed form.
"""
from __future__ import annotations

import math
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle
import valueround as vr
from test_oracle_pack import NTHREADS, run_checker, structured_inputs

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("chkm") / "value_check")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-o", exe,
                    os.path.join(HERE, "checker", "value_check.c"), "-ldl", "-lpthread", "-lm"], check=True)
    return exe


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


@pytest.mark.parametrize("k,mode", [(2, 1), (2, 2), (3, 2)])
def test_value_checker_modes_exhaustive(checker, k, mode):
    rc, out = run_checker(checker, oracle.lib_path(0), k, 0, 0, NTHREADS, mode)
    assert rc == 0 and "checked=4294967296 mismatches=0" in out, out


def test_value_checker_toward_zero_k3_sample(checker):
    rc, out = run_checker(checker, oracle.lib_path(0), 3, 0x3E000000, 1 << 26, NTHREADS, 1)
    assert rc == 0, out
    rc, out = run_checker(checker, oracle.lib_path(0), 3, 0x80000000, 1 << 24, NTHREADS, 1)
    assert rc == 0, out


def test_boldo_melquiond_property_exhaustive(checker):
    rc, out = run_checker(checker, oracle.lib_path(0), "bm", 2, 3, NTHREADS)
    assert rc == 0 and "mismatches=0" in out, out


def read_modes_table():
    rows = []
    for line in open(os.path.join(HERE, "golden", "pack_modes_table.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            p = line.split(None, 5)
            rows.append((int(p[0]), int(p[1]), int(p[2]), int(p[3], 16), int(p[4], 16), p[5] if len(p) > 5 else ""))
    return rows


def test_modes_golden_table(orc):
    rows = read_modes_table()
    assert len(rows) >= 20
    for b, k, mode, u, want, why in rows:
        assert orc.pack_bits_mode(b, k, u, mode) == want, (b, k, mode, hex(u), why)
        e = vr.expected_pack_mode(b, k, u, mode)
        if e is not None:
            assert e == want, (b, k, mode, hex(u), hex(e), why)


@pytest.mark.parametrize("base,k", oracle.FORMATS)
@pytest.mark.parametrize("mode", [1, 2])
def test_modes_structured_sweep(orc, base, k, mode):
    for u in structured_inputs(base, k):
        got = orc.pack_bits_mode(base, k, u, mode)
        want = vr.expected_pack_mode(base, k, u, mode)
        if want is None:
            assert vr.decode(base, orc.unpack_bits(base, k, got)) == "nan"
        else:
            assert got == want, (base, k, mode, hex(u), hex(got), hex(want))


def test_mode_zero_is_nearest_even(orc):
    for b, k in oracle.FORMATS:
        for u in structured_inputs(b, k)[::7]:
            assert orc.pack_bits_mode(b, k, u, 0) == orc.pack_bits(b, k, u)


def test_planted_round_to_odd_mutation_is_caught(checker):
    oracle.build(6)
    m = oracle.Oracle(6)
    assert any(m.pack_bits_mode(b, k, u, mode) != w for b, k, mode, u, w, _ in read_modes_table())
    rc, _ = run_checker(checker, oracle.lib_path(6), "bm", 2, 3, NTHREADS)
    assert rc != 0


# ---------------------------------------------------------------- scale and magnitude
def wide(n, seed, base):
    g = np.random.default_rng(seed)
    if base == 32:
        return (g.standard_normal(n) * np.exp2(g.uniform(-30, 30, n))).astype(np.float32)
    return g.standard_normal(n) * np.exp2(g.uniform(-200, 200, n))


@pytest.mark.parametrize("base,k", oracle.FORMATS)
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_scale_vs_rational(orc, base, k, mode):
    n = 300
    x = orc.pack(base, k, wide(n, 31 + k, base))
    alpha = float.fromhex("0x1.5555555555555p-2")
    got = orc.scale(base, k, alpha, x, mode)
    a = Fraction(float(np.float32(alpha))) if base == 32 else Fraction(alpha)
    xs = orc.unpack(base, k, x).view(np.uint32 if base == 32 else np.uint64)
    gu = orc.unpack(base, k, got).view(np.uint32 if base == 32 else np.uint64)
    E, m, bias, emin, emax = vr.params(base, k)
    for i in range(n):
        xv = vr.decode(base, int(xs[i]))
        r = vr.round_to_base(a * xv, base)
        neg = (r == vr.NINF) or (r not in (vr.INF, vr.NINF) and r < 0) or (r == 0 and xv < 0)
        if r in (vr.INF, vr.NINF):
            want = vr.encode(base, k, r, neg)
        elif mode == 0:
            want = vr.encode(base, k, vr.round_rne(r, m + 1, emin, emax), neg)
        else:
            want = vr.encode(base, k, vr.round_directed(r, m + 1, emin, mode), neg)
        q = orc.pack_bits_mode(base, k, int(gu[i]), 0)   # back to the k-byte integer (exact: on the grid)
        assert q == want, (base, k, mode, i)


@pytest.mark.parametrize("base,k", [(32, 2), (32, 3), (64, 3), (64, 5), (64, 8)])
def test_nrm2_exact_vs_rational(orc, base, k):
    x = orc.pack(base, k, wide(400, 41 + k, base))
    xs = [vr.decode(base, int(u)) for u in orc.unpack(base, k, x).view(np.uint32 if base == 32 else np.uint64)]
    s2 = vr.round_to_base(sum((v * v for v in xs), Fraction(0)), base)
    want = math.sqrt(float(s2)) if base == 64 else float(np.sqrt(np.float32(float(s2))))
    assert orc.nrm2_exact(base, k, x) == want


def test_nrm2_naive_closed_form(orc):
    x = orc.pack(64, 5, np.array([3.0, 4.0, 12.0, 84.0]))
    assert orc.nrm2_naive(64, 5, x) == 85.0          # 9 + 16 + 144 + 7056 = 7225 = 85^2
    x = orc.pack(32, 3, np.array([2.0 ** 60, 2.0 ** 60], dtype=np.float32))
    assert orc.nrm2_naive(32, 3, x) == float(np.float32(2.0 ** 60 * math.sqrt(2.0)))
