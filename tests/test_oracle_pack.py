"""Pins of the oracle's pack/unpack (C1, C2) against things other than itself.

* a hand-built table of rounding cases (tests/golden/pack_rne_table.txt);
* an independent value-domain checker, exhaustive on all 2^32 binary32 inputs
  for k = 2 and k = 3 (tests/checker/value_check.c);
* a library special case: binary32 k = 2 is bfloat16, and torch's CPU
  float32 -> bfloat16 conversion rounds to nearest even;
* exact rational rounding (fractions) on structured sweeps and random inputs
  for every format, including the binary64 ones;
* exhaustive round trips pack(unpack(q)) == q where the pattern space allows;
* invariants (idempotence, sign symmetry, monotonicity, half-ulp bound, NaN in
  iff NaN out) with hypothesis;
* the paper's add-half-ULP heuristic as a negative control, and planted
  mutations of the oracle that the pins above must catch.
"""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
import valueround as vr
from paper_1601_07789_amd import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "pack_rne_table.txt")
FORMATS = oracle.FORMATS
NTHREADS = max(1, min(16, os.cpu_count() or 1))


def read_table():
    rows = []
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split(None, 4)
            rows.append((int(parts[0]), int(parts[1]), int(parts[2], 16), int(parts[3], 16),
                         parts[4] if len(parts) > 4 else ""))
    return rows


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("chk") / "value_check")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-o", exe,
                    os.path.join(HERE, "checker", "value_check.c"), "-ldl", "-lpthread", "-lm"],
                   check=True)
    return exe


def run_checker(exe, so, *args):
    r = subprocess.run([exe, so, *map(str, args)], capture_output=True, text=True)
    return r.returncode, r.stdout


# ---------------------------------------------------------------- golden table
def test_golden_table(orc):
    rows = read_table()
    assert len(rows) >= 50
    bad = [(b, k, hex(u), hex(want), hex(orc.pack_bits(b, k, u)), why)
           for b, k, u, want, why in rows if orc.pack_bits(b, k, u) != want]
    assert not bad, bad


def test_golden_table_agrees_with_value_rounding():
    """The table itself against exact rational rounding (non-NaN rows)."""
    for b, k, u, want, why in read_table():
        e = vr.expected_pack(b, k, u)
        if e is not None:
            assert e == want, (b, k, hex(u), hex(want), hex(e), why)


def test_format_table(orc):
    """Table 1 field widths (sign/exponent/mantissa) and the m = 8k-1-E rule."""
    table1 = {(32, 2): 7, (32, 3): 15, (32, 4): 23, (64, 5): 28, (64, 6): 36, (64, 7): 44, (64, 8): 52}
    for f, m in table1.items():
        assert orc.mant_bits(*f) == m
    for k, m in [(2, 4), (3, 12), (4, 20)]:
        assert orc.mant_bits(64, k) == m
    lib = oracle.load()
    assert not lib.fbo_format_valid(32, 1) and not lib.fbo_format_valid(32, 5)
    assert not lib.fbo_format_valid(64, 1) and not lib.fbo_format_valid(64, 9)
    assert not lib.fbo_format_valid(16, 2)


# ---------------------------------------------------------------- exhaustive binary32
@pytest.mark.parametrize("k", [2, 3])
def test_value_checker_exhaustive_binary32(checker, k):
    rc, out = run_checker(checker, oracle.lib_path(0), k, 0, 0, NTHREADS)
    assert rc == 0, out
    assert "checked=4294967296 mismatches=0" in out


@pytest.mark.parametrize("base,k", [(32, 2), (32, 3), (64, 2), (64, 3), (64, 4)])
def test_round_trip_exhaustive(checker, base, k):
    rc, out = run_checker(checker, oracle.lib_path(0), "rt", base, k, NTHREADS)
    assert rc == 0, out
    assert f"checked={1 << (8 * k)} mismatches=0" in out


def test_bf16_library_special_case(orc):
    """binary32 k=2 is bfloat16: every non-NaN input must match torch's RNE conversion."""
    torch = pytest.importorskip("torch")
    from concurrent.futures import ThreadPoolExecutor
    chunk = 1 << 24

    def one(start):
        u = np.arange(start, start + chunk, dtype=np.uint64).astype(np.uint32)
        ref = torch.from_numpy(u.view(np.float32)).to(torch.bfloat16).view(torch.int16).numpy()
        got = orc.pack(32, 2, u).view(np.int16)
        nan = (u & 0x7FFFFFFF) > 0x7F800000
        bad = np.nonzero((ref != got) & ~nan)[0]
        return [(hex(int(u[i])), hex(int(got[i]) & 0xFFFF), hex(int(ref[i]) & 0xFFFF)) for i in bad[:5]]

    torch.set_num_threads(1)
    with ThreadPoolExecutor(NTHREADS) as ex:
        bad = [b for r in ex.map(one, range(0, 1 << 32, chunk)) for b in r]
    assert not bad, bad[:10]


# ---------------------------------------------------------------- rational rounding, all formats
def structured_inputs(base: int, k: int):
    """sign x exponent x kept mantissa x dropped bits, covering every branch."""
    E = 8 if base == 32 else 11
    M = base - 1 - E
    d = base - 8 * k
    m = M - d
    maxe = (1 << E) - 1
    exps = sorted({0, 1, 2, (1 << (E - 1)) - 1, maxe - 2, maxe - 1, maxe})
    g = np.random.default_rng(7 + base + k)
    kept = sorted({0, 1, 2, (1 << m) - 2, (1 << m) - 1, int(g.integers(0, 1 << m))})
    if d == 0:
        drops = [0]
    else:
        half = 1 << (d - 1)
        drops = sorted({0, 1, half - 1, half, half + 1, (1 << d) - 1, int(g.integers(0, 1 << d))})
    out = []
    for s in (0, 1):
        for e in exps:
            for km in kept:
                for dr in drops:
                    out.append((s << (base - 1)) | (e << M) | (km << d) | dr)
    return out


@pytest.mark.parametrize("base,k", FORMATS)
def test_structured_sweep_vs_rational_rounding(orc, base, k):
    for u in structured_inputs(base, k):
        got = orc.pack_bits(base, k, u)
        want = vr.expected_pack(base, k, u)
        if want is None:       # NaN: must stay NaN with the same sign
            back = orc.unpack_bits(base, k, got)
            assert vr.decode(base, back) == "nan", hex(u)
            assert back >> (base - 1) == u >> (base - 1)
        else:
            assert got == want, (base, k, hex(u), hex(got), hex(want))


@pytest.mark.parametrize("k", range(2, 9))
def test_mixed_population_vs_rational_rounding(orc, k):
    bits = workloads.mixed_binary64(4000, workloads.SEED_BASE)
    got = orc.pack_u64(64, k, bits)
    for u, q in zip(bits.tolist(), got.tolist()):
        want = vr.expected_pack(64, k, u)
        if want is None:
            assert vr.decode(64, orc.unpack_bits(64, k, q)) == "nan"
        else:
            assert q == want, (k, hex(u), hex(q), hex(want))


# ---------------------------------------------------------------- invariants
def _as_signed_order(base, u):
    """Map a non-NaN pattern to an integer that orders like its value."""
    sign = u >> (base - 1)
    mag = u & ((1 << (base - 1)) - 1)
    return -mag if sign else mag


@settings(max_examples=3000, deadline=None)
@given(fmt=st.sampled_from(FORMATS), u=st.integers(min_value=0, max_value=(1 << 64) - 1),
       v=st.integers(min_value=0, max_value=(1 << 64) - 1))
def test_invariants(fmt, u, v):
    orc = oracle.default()
    base, k = fmt
    u &= (1 << base) - 1
    v &= (1 << base) - 1
    q = orc.pack_bits(base, k, u)
    back = orc.unpack_bits(base, k, q)
    # idempotence: pack(unpack(pack(x))) == pack(x)
    assert orc.pack_bits(base, k, back) == q
    # sign symmetry
    sbit = 1 << (base - 1)
    assert orc.pack_bits(base, k, u ^ sbit) == q ^ (1 << (8 * k - 1))
    nan_in = vr.decode(base, u) == "nan"
    nan_out = vr.decode(base, back) == "nan"
    assert nan_in == nan_out
    if nan_in:
        return
    # result is one of the two grid neighbours (truncation or truncation + 1 ulp)
    d = base - 8 * k
    trunc = u >> d
    assert q in (trunc, trunc + 1)
    # |unpack(pack(x)) - x| <= half an ulp of the format (finite results)
    xv, rv = vr.decode(base, u), vr.decode(base, back)
    if xv not in (vr.INF, vr.NINF) and rv not in (vr.INF, vr.NINF):
        _, m, _, emin, _ = vr.params(base, k)
        a = abs(xv)
        e = vr.floor_log2(a) if a else emin
        ulp = vr.Fraction(2) ** (max(e, emin) - m)
        assert abs(rv - xv) <= ulp / 2
    # monotonicity on ordered non-NaN inputs
    if vr.decode(base, v) != "nan":
        qv = orc.pack_bits(base, k, v)
        if _as_signed_order(base, u) <= _as_signed_order(base, v):
            a1 = vr.decode(base, back)
            a2 = vr.decode(base, orc.unpack_bits(base, k, qv))
            key = lambda z: (-1, 0) if z == vr.NINF else ((1, 0) if z == vr.INF else (0, z))
            assert key(a1) <= key(a2)


# ---------------------------------------------------------------- negative control and mutations
def test_heuristic_negative_control():
    """The add-half-ULP heuristic must disagree with round-to-nearest-even on ties and NaNs."""
    heur = oracle.Oracle(3)
    real = oracle.default()
    ties = [(32, 2, 0x3F808000), (32, 2, 0xBF808000), (32, 2, 0x00008000), (32, 3, 0x3F800080),
            (64, 5, 0x3FF0000000800000), (64, 2, 0x3FF0800000000000)]
    for b, k, u in ties:
        assert heur.pack_bits(b, k, u) != real.pack_bits(b, k, u), hex(u)
    assert heur.pack_bits(32, 2, 0x7FFFFFFF) == 0x8000     # NaN overflows into the sign
    assert real.pack_bits(32, 2, 0x7FFFFFFF) == 0x7FFF
    table = read_table()
    assert any(heur.pack_bits(b, k, u) != want for b, k, u, want, _ in table)


def _pins_pass(mut: int, checker) -> bool:
    o = oracle.Oracle(mut)
    for b, k, u, want, _ in read_table():
        if o.pack_bits(b, k, u) != want:
            return False
    for base, k in [(32, 2), (64, 3)]:
        rc, _ = run_checker(checker, oracle.lib_path(mut), "rt", base, k, NTHREADS)
        if rc != 0:
            return False
    rc, _ = run_checker(checker, oracle.lib_path(mut), 2, 0xBF000000, 1 << 22, NTHREADS)
    return rc == 0


@pytest.mark.parametrize("mut", [1, 2, 3, 4, 5])
def test_planted_mutation_is_caught(checker, mut):
    oracle.build(mut)
    assert oracle.Oracle(mut).lib.fbo_mutation() == mut
    assert not _pins_pass(mut, checker)


def test_real_oracle_passes_the_same_pins(checker):
    assert _pins_pass(0, checker)
