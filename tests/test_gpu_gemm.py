"""GPU parity of fb_gemm against the exact oracle.

Error measures (componentwise-normwise, so near-zero entries do not blow up):
  e1 = max_ij |C_ij - C*_ij| / (|A||B|)_ij
Bounds (K inner dimension, u32 = 2^-24, u64 = 2^-53, gamma_n(u) = n u / (1 - n u)):
  BF16 ({32,2}):      products exact in FP32        -> e1 <= gamma_K(u32)
  3-product ({32,3}): |lo| < 2^-7 |x|, lo*lo dropped -> e1 <= 2^-14 + gamma_3K(u32) (1 + 2^-7)^2
  4-product:          every product exact          -> e1 <= gamma_4K(u32) (1 + 2^-7)^2
  FP64 ({64,2..8}):   |unpack(C) - C*| <= gamma_K(u64) (|A||B|) + 2^-(m+1) (|C*| + gamma_K(u64) (|A||B|))
  scaled pieces ({64,2..4} on BF16 matrix cores, P = k - 1 pieces of 8, 8, 5 bits,
  |piece_i| < 2^-7i |x|): e1 <= drop + gamma_{nK}(u32) (1 + 2^-7 + 2^-14)^2, n the
  number of products formed (1; 3 or 4; 6 or 9), drop the bound of the products
  left out (0; 2^-14; 2^-20 (1 + 2^-8)), then the cut to the output format.
Integer-valued data whose products and sums are exact in the accumulation
type must give C (or the oracle's pack of it) bit for bit.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_helpers import device, log
from paper_1601_07789_amd import flyte, workloads

pytestmark = pytest.mark.gpu

U32, U64 = 2.0 ** -24, 2.0 ** -53


def gam(n, u):
    return n * u / (1 - n * u)


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


def all_entries(M, N):
    ii, jj = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
    return ii.reshape(-1), jj.reshape(-1)


@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("shape", [(256, 384, 320), (512, 512, 192), (128, 256, 64)])
def test_gemm_binary32_small_all_entries(dev, orc, k, shape):
    """Every entry; the shapes exercise the 256 x 256, 256 x 128 and 128 x 128 tile paths.
    k = 4 here means the 3-byte operands with the four-product option."""
    import torch
    log(f"gemm b32 k={k} {shape}")
    four = k == 4
    k = 3 if four else k
    M, N, K = shape
    g = np.random.default_rng(11 + k)
    Av = g.standard_normal((M, K)).astype(np.float32)
    Bv = g.standard_normal((K, N)).astype(np.float32)
    # a few rows/columns spanning a wide exponent range
    Av[3] *= np.float32(2.0 ** 20)
    Bv[:, 5] *= np.float32(2.0 ** -20)
    A, B = orc.pack(32, k, Av.reshape(-1)), orc.pack(32, k, Bv.reshape(-1))
    C = flyte.gemm((32, k), (32, k), (32, 4), M, N, K, torch.from_numpy(A).to(dev),
                   torch.from_numpy(B).to(dev), flags=flyte.GEMM_FOUR_PRODUCTS if four else 0)
    C = C.cpu().numpy().reshape(M, N).astype(np.float64)
    ii, jj = all_entries(M, N)
    ce, cab = orc.gemm_entries((32, k), (32, k), K, A, K, B, N, ii, jj)
    e1 = np.max(np.abs(C.reshape(-1) - ce) / cab)
    if four:
        bound = gam(4 * K, U32) * (1 + 2.0 ** -7) ** 2
    else:
        bound = gam(K, U32) if k == 2 else 2.0 ** -14 + gam(3 * K, U32) * (1 + 2.0 ** -7) ** 2
    assert e1 <= bound, (e1, bound)
    if k == 3:
        # the 3-product must be far more accurate than plain BF16 of the rounded inputs
        assert e1 < 2.0 ** -12


@pytest.mark.parametrize("shape", [(256, 256, 64), (256, 384, 64), (128, 128, 64), (384, 128, 64)])
def test_gemm_split_products_exact_construction(dev, orc, shape):
    """{32,3} operands on which every split product and partial sum is exact in
    binary32 (split_exact): four products must give the exact C bit for bit and
    three products the exact C minus sum_k lo*lo, bit for bit.  A kernel that
    dropped or added any one product fails (tests/test_split_model.py)."""
    import torch
    import split_exact
    log(f"gemm split products exact {shape}")
    M, N, K = shape
    Av = split_exact.values(M, K, 40 + M, 1)
    Bv = split_exact.values(K, N, 41 + N, 0)
    A, B = orc.pack(32, 3, Av.reshape(-1)), orc.pack(32, 3, Bv.reshape(-1))
    ii, jj = all_entries(M, N)
    exact, _ = orc.gemm_entries((32, 3), (32, 3), K, A, K, B, N, ii, jj)
    exact = exact.reshape(M, N)
    _, Al = split_exact.split(Av)
    _, Bl = split_exact.split(Bv)
    lolo = Al @ Bl
    assert np.any(lolo != 0)
    Ad, Bd = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    for four, want in ((True, exact), (False, exact - lolo)):
        C = flyte.gemm((32, 3), (32, 3), (32, 4), M, N, K, Ad, Bd,
                       flags=flyte.GEMM_FOUR_PRODUCTS if four else 0).cpu().numpy().reshape(M, N)
        assert np.array_equal(C.astype(np.float64), want), (four, int(np.sum(C != want)))


def test_gemm_f64_integer_data_bit_exact(dev, orc):
    import torch
    log("gemm f64 integer")
    M, N, K = 256, 256, 192
    g = np.random.default_rng(5)
    for kin in (2, 3, 4, 5, 6, 7, 8):
        lim = 31 if kin == 2 else 64           # {64,2} holds integers up to 2^5 - 1 exactly
        Av = g.integers(-lim, lim + 1, (M, K)).astype(np.float64)
        Bv = g.integers(-lim, lim + 1, (K, N)).astype(np.float64)
        exact = Av @ Bv                        # exact: |C| < 2^20
        A, B = orc.pack(64, kin, Av.reshape(-1)), orc.pack(64, kin, Bv.reshape(-1))
        Ad, Bd = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
        for kout in (2, 3, 4, 5, 6, 7, 8):
            C = flyte.gemm((64, kin), (64, kin), (64, kout), M, N, K, Ad, Bd).cpu().numpy()
            want = orc.pack(64, kout, exact.reshape(-1))
            assert np.array_equal(C if kout < 8 else C.view(np.uint8), want), (kin, kout)


@pytest.mark.parametrize("kin,kout", [(5, 5), (6, 6), (5, 8), (6, 3), (2, 2), (3, 3), (4, 4), (2, 8), (4, 6), (7, 7),
                                      (8, 8), (8, 5)])
def test_gemm_f64_random_all_entries(dev, orc, kin, kout):
    """The FP64 matrix-core path (the only one for k >= 5; FB_GEMM_FP64 for k <= 4),
    rows of A scaled over 2^-300 .. 2^300: the full binary64 exponent range."""
    import torch
    log(f"gemm f64 {kin}->{kout}")
    M, N, K = 128, 256, 208
    g = np.random.default_rng(7 + kin + kout)
    Av = g.standard_normal((M, K)) * np.exp2(np.round(g.uniform(-300, 300, (M, 1))))
    Bv = g.standard_normal((K, N))
    A, B = orc.pack(64, kin, Av.reshape(-1)), orc.pack(64, kin, Bv.reshape(-1))
    C = flyte.gemm((64, kin), (64, kin), (64, kout), M, N, K, torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev),
                   flags=flyte.GEMM_FP64)
    Cu = orc.unpack(64, kout, C.cpu().numpy().view(np.uint8)) if kout < 8 else C.cpu().numpy()
    ii, jj = all_entries(M, N)
    ce, cab = orc.gemm_entries((64, kin), (64, kin), K, A, K, B, N, ii, jj)
    m = 8 * kout - 12
    bound = gam(K, U64) * cab + 2.0 ** -(m + 1) * (np.abs(ce) + gam(K, U64) * cab)
    err = np.abs(Cu.reshape(-1) - ce)
    assert np.all(err <= bound * (1 + 1e-12)), np.max(err / np.maximum(bound, 1e-300))


def test_gemm_k_zero_gives_zero(dev):
    import torch
    A = torch.zeros(16, dtype=torch.uint8, device=dev)
    B = torch.zeros(128 * 5, dtype=torch.uint8, device=dev)
    C = torch.full((128 * 128 * 5,), 0x77, dtype=torch.uint8, device=dev)
    flyte.gemm((64, 5), (64, 5), (64, 5), 128, 128, 0, A, B, C=C, lda=4, ldb=128)
    assert torch.all(C == 0).item()


def sampled(orc, fa, K, A, B, N, C, M, seed, count=256):
    rng = np.random.default_rng(seed)
    ii = np.concatenate([[0, M - 1], rng.integers(0, M, count)])
    jj = np.concatenate([[0, N - 1], rng.integers(0, N, count)])
    ce, cab = orc.gemm_entries(fa, fa, K, A, K, B, N, ii, jj)
    return ii, jj, ce, cab


@pytest.mark.parametrize("k", [2, 3])
def test_gemm_binary32_benchmark_size_sampled(dev, orc, k):
    """M = N = K = 8192, N(0,1) entries (the precision-GEMM workload): sampled entries.
    For {32,3} both the three- and the four-product GEMM run on the same operands;
    each meets its bound, and adding lo*lo must at least halve e1 (the dropped term
    is the three-product's main error on this data)."""
    import torch
    log(f"gemm b32 k={k} 8192^3 sampled")
    n = 8192
    g = torch.Generator(device=dev)
    g.manual_seed(workloads.SEED_BASE + 2)
    v = torch.empty(n * n, dtype=torch.float32, device=dev).normal_(generator=g)
    A = flyte.pack((32, k), v)
    v.normal_(generator=g)
    B = flyte.pack((32, k), v)
    del v
    Ah, Bh = A.cpu().numpy(), B.cpu().numpy()
    ii, jj, ce, cab = sampled(orc, (32, k), n, Ah, Bh, n, None, n, 3)
    e1 = {}
    for four in ((False, True) if k == 3 else (False,)):
        C = flyte.gemm((32, k), (32, k), (32, 4), n, n, n, A, B, flags=flyte.GEMM_FOUR_PRODUCTS if four else 0)
        torch.cuda.synchronize()
        got = C.view(n, n)[torch.from_numpy(ii).to(dev), torch.from_numpy(jj).to(dev)].cpu().numpy()
        e1[four] = np.max(np.abs(got.astype(np.float64) - ce) / cab)
        if four:
            bound = gam(4 * n, U32) * (1 + 2.0 ** -7) ** 2
        else:
            bound = gam(n, U32) if k == 2 else 2.0 ** -14 + gam(3 * n, U32) * (1 + 2.0 ** -7) ** 2
        log(f"  four={four} e1 = {e1[four]:.3e} (bound {bound:.3e})")
        assert e1[four] <= bound
        del C
    if k == 3:
        assert e1[True] < e1[False] / 2, e1
    del A, B
    torch.cuda.empty_cache()


@pytest.mark.parametrize("k", [5, 6, 3])
def test_gemm_f64_benchmark_size_sampled(dev, orc, k):
    """M = N = K = 16384, N(0,1) entries, C packed to the same k: sampled entries."""
    import torch
    log(f"gemm f64 k={k} 16384^3 sampled")
    n = 16384
    g = torch.Generator(device=dev)
    g.manual_seed(workloads.SEED_BASE + 4)
    v = torch.empty(n * n, dtype=torch.float64, device=dev).normal_(generator=g)
    A = flyte.pack((64, k), v)
    v.normal_(generator=g)
    B = flyte.pack((64, k), v)
    del v
    C = flyte.gemm((64, k), (64, k), (64, k), n, n, n, A, B, flags=flyte.GEMM_FP64 if k <= 4 else 0)
    torch.cuda.synchronize()
    Ah, Bh = A.cpu().numpy(), B.cpu().numpy()
    ii, jj, ce, cab = sampled(orc, (64, k), n, Ah, Bh, n, None, n, 4, count=128)
    idx = torch.from_numpy(((ii * n + jj)[:, None] * k + np.arange(k)[None, :]).reshape(-1)).to(dev)
    got = orc.unpack(64, k, C[idx].cpu().numpy())
    m = 8 * k - 12
    bound = gam(n, U64) * cab + 2.0 ** -(m + 1) * (np.abs(ce) + gam(n, U64) * cab)
    assert np.all(np.abs(got - ce) <= bound * (1 + 1e-12))
    del A, B, C
    torch.cuda.empty_cache()


def _special_entries(orc, fa, K, A, B, N, M):
    ii, jj = all_entries(M, N)
    return orc.gemm_entries(fa, fa, K, A, K, B, N, ii, jj)


def test_gemm_bf16_subnormal_operands(dev, orc):
    """{32,2} rows of A made of bfloat16 subnormals (m * 2^-133) against B ~ 2^60..2^90, so
    every product is a normal binary32 number: the products stay exact only if the matrix
    cores keep subnormal inputs (a flush would zero those rows, e1 ~ 1)."""
    import torch
    M, N, K = 128, 128, 64
    g = np.random.default_rng(21)
    Av = (g.standard_normal((M, K)) * np.exp2(np.round(g.uniform(-20, 10, (M, 1))))).astype(np.float32)
    sub = (g.integers(1, 128, (M // 2, K)) * g.choice([-1.0, 1.0], (M // 2, K))).astype(np.float64) * 2.0 ** -133
    Av[M // 2:] = sub.astype(np.float32)
    Bv = (g.standard_normal((K, N)) * np.exp2(np.round(g.uniform(60, 90, (1, N))))).astype(np.float32)
    A, B = orc.pack(32, 2, Av.reshape(-1)), orc.pack(32, 2, Bv.reshape(-1))
    assert np.array_equal(orc.unpack(32, 2, A).reshape(M, K)[M // 2:], Av[M // 2:])   # exactly bfloat16
    C = flyte.gemm((32, 2), (32, 2), (32, 4), M, N, K, torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev))
    C = C.cpu().numpy().astype(np.float64)
    ce, cab = _special_entries(orc, (32, 2), K, A, B, N, M)
    e1 = np.abs(C - ce) / cab
    assert np.max(e1[: M * N // 2]) <= gam(K, U32)
    assert np.max(e1[M * N // 2:]) <= gam(K, U32), "subnormal bfloat16 inputs were not kept"


def test_gemm_f64_subnormal_operands(dev, orc):
    """{64,5} rows of A made of binary64 subnormals (~2^-1060) against B ~ 2^100: products
    are normal, so FP64 matrix cores that keep subnormal inputs stay within the bound."""
    import torch
    M, N, K = 128, 128, 64
    g = np.random.default_rng(22)
    Av = g.standard_normal((M, K))
    Av[M // 2:] *= 2.0 ** -1060
    Bv = g.standard_normal((K, N)) * 2.0 ** 100
    A, B = orc.pack(64, 5, Av.reshape(-1)), orc.pack(64, 5, Bv.reshape(-1))
    C = flyte.gemm((64, 5), (64, 5), (64, 8), M, N, K, torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev))
    ce, cab = _special_entries(orc, (64, 5), K, A, B, N, M)
    err = np.abs(C.cpu().numpy().reshape(-1) - ce)
    assert np.all(err <= gam(K, U64) * cab * (1 + 1e-12) + 2.0 ** -1074)


@pytest.mark.parametrize("case", ["bf16", "three", "four", "f64"])
def test_gemm_special_values(dev, orc, case):
    """Inf, -Inf and NaN operands (and zeros beside them): entries whose exact value is NaN
    are NaN, finite ones meet the bound.  Exact infinities are reproduced by the BF16 and
    FP64 paths; the split products give NaN or the infinity, since the hi*lo term of an
    infinite element's partner can be Inf * 0."""
    import torch
    M, N, K = 128, 128, 64
    g = np.random.default_rng(23)
    base, k = (64, 5) if case == "f64" else (32, 2 if case == "bf16" else 3)
    dt = np.float64 if base == 64 else np.float32
    Av = g.standard_normal((M, K)).astype(dt)
    Bv = g.standard_normal((K, N)).astype(dt)
    Av[3, 5], Av[70, 9], Av[100, 40] = np.inf, -np.inf, np.nan
    if base == 32:
        # a NaN whose kept payload lies only in the low byte ({32,3} pattern 7F8001; for
        # {32,2} the pattern rounds to 7F80|quiet bit): every entry of row 110 is NaN
        Av[110, 17] = np.array([0x7F800100], dtype=np.uint32).view(np.float32)[0]
    Bv[5, 7] = 0.0             # Inf * 0 in entry (3, 7)
    Bv[11, 100] = np.inf       # row 11 of B meets every row of A
    Bv[12, 100] = -np.inf      # Inf - Inf in column 100
    Bv[20, 50] = np.nan
    A, B = orc.pack(base, k, Av.reshape(-1)), orc.pack(base, k, Bv.reshape(-1))
    fc = (64, 8) if base == 64 else (32, 4)
    flags = flyte.GEMM_FOUR_PRODUCTS if case == "four" else 0
    C = flyte.gemm((base, k), (base, k), fc, M, N, K, torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev),
                   flags=flags).cpu().numpy().astype(np.float64).reshape(-1)
    ce, cab = _special_entries(orc, (base, k), K, A, B, N, M)
    nan, inf = np.isnan(ce), np.isinf(ce)
    assert nan.sum() > 0 and inf.sum() > 0
    assert np.all(np.isnan(C[nan]))
    if case in ("bf16", "f64"):
        assert np.array_equal(C[inf], ce[inf])
    else:
        assert np.all(np.isnan(C[inf]) | (C[inf] == ce[inf]))
    fin = ~(nan | inf)
    if case == "bf16":
        bound = gam(K, U32)
    elif case == "three":
        bound = 2.0 ** -14 + gam(3 * K, U32) * (1 + 2.0 ** -7) ** 2
    elif case == "four":
        bound = gam(4 * K, U32) * (1 + 2.0 ** -7) ** 2
    else:
        bound = gam(K, U64)
    assert np.all(np.isfinite(C[fin]))
    assert np.max(np.abs(C[fin] - ce[fin]) / cab[fin]) <= bound


@pytest.mark.parametrize("case", ["bf16", "three", "four", "f64"])
def test_gemm_padded_leading_dimensions(dev, orc, case):
    """lda > K, ldb > N, ldc > N (rows padded, still 4-byte aligned): every entry within the
    bound, and C's padding columns untouched."""
    import torch
    M, N, K = 256, 256, 128
    base, k = (64, 5) if case == "f64" else (32, 2 if case == "bf16" else 3)
    lda, ldb, ldc = K + 4, N + 8, N + 4
    g = np.random.default_rng(31)
    dt = np.float64 if base == 64 else np.float32
    Av = g.standard_normal((M, lda)).astype(dt)
    Bv = g.standard_normal((K, ldb)).astype(dt)
    A, B = orc.pack(base, k, Av.reshape(-1)), orc.pack(base, k, Bv.reshape(-1))
    if base == 64:
        fc, cdt, kc = (64, 8), torch.float64, 8
    else:
        fc, cdt, kc = (32, 4), torch.float32, 4
    C = torch.full((M * ldc,), 7.0, dtype=cdt, device=dev)
    flags = flyte.GEMM_FOUR_PRODUCTS if case == "four" else 0
    flyte.gemm((base, k), (base, k), fc, M, N, K, torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev), C=C,
               lda=lda, ldb=ldb, ldc=ldc, flags=flags)
    Ch = C.cpu().numpy().reshape(M, ldc).astype(np.float64)
    assert np.all(Ch[:, N:] == 7.0)
    ii, jj = all_entries(M, N)
    ce, cab = orc.gemm_entries((base, k), (base, k), K, A, lda, B, ldb, ii, jj)
    e1 = np.max(np.abs(Ch[:, :N].reshape(-1) - ce) / cab)
    bound = {"bf16": gam(K, U32), "three": 2.0 ** -14 + gam(3 * K, U32) * (1 + 2.0 ** -7) ** 2,
             "four": gam(4 * K, U32) * (1 + 2.0 ** -7) ** 2, "f64": gam(K, U64)}[case]
    assert e1 <= bound, (e1, bound)


# ---------------------------------------------------------------- shapes that are not tile multiples
def _ld(n, k):
    g = {1: 4, 2: 2, 3: 4, 4: 1, 5: 4, 6: 2, 7: 4, 8: 1}[k]
    return (n + g - 1) // g * g        # rows start 4-byte aligned


# the last two: N a multiple of 4 and K of 32 (edge rows and column groups clamped in the piece kernel)
RAGGED = [(300, 310, 277), (1, 5, 3), (129, 257, 65), (300, 200, 4), (257, 131, 1), (300, 260, 96), (1, 4, 32)]


@pytest.mark.parametrize("case", ["bf16", "three", "four"])
@pytest.mark.parametrize("shape", RAGGED)
def test_gemm_ragged_binary32(dev, orc, case, shape):
    """M, N, K not tile multiples (and K below one step): every entry within the
    bound, C's padding columns untouched."""
    import torch
    log(f"gemm ragged {case} {shape}")
    M, N, K = shape
    k = 2 if case == "bf16" else 3
    lda, ldb, ldc = _ld(K, k) + (4 if k == 3 else 2), _ld(N, k), N + 3
    g = np.random.default_rng(M * 7 + N + K)
    A = orc.pack(32, k, g.standard_normal(M * lda).astype(np.float32))
    B = orc.pack(32, k, g.standard_normal(K * ldb).astype(np.float32))
    C = torch.full((M * ldc,), 7.0, dtype=torch.float32, device=dev)
    flyte.gemm((32, k), (32, k), (32, 4), M, N, K, torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev), C=C,
               lda=lda, ldb=ldb, ldc=ldc, flags=flyte.GEMM_ALL_PRODUCTS if case == "four" else 0)
    Ch = C.cpu().numpy().reshape(M, ldc).astype(np.float64)
    assert np.all(Ch[:, N:] == 7.0)
    ii, jj = all_entries(M, N)
    ce, cab = orc.gemm_entries((32, k), (32, k), K, A, lda, B, ldb, ii, jj)
    bound = {"bf16": gam(K, U32), "three": 2.0 ** -14 + gam(3 * K, U32) * (1 + 2.0 ** -7) ** 2,
             "four": gam(4 * K, U32) * (1 + 2.0 ** -7) ** 2}[case]
    assert np.all(np.abs(Ch[:, :N].reshape(-1) - ce) <= bound * cab)


@pytest.mark.parametrize("case,shape", [("bf16", (4100, 4104, 333)), ("bf16", (4097, 4099, 70)),
                                        ("three", (4100, 4104, 320)), ("four", (4100, 4104, 320)),
                                        ("three", (4097, 4099, 70)), ("four", (4100, 4104, 333))])
def test_gemm_bf16_large_edges(dev, orc, case, shape):
    """Shapes large enough for 256 x 256 tiles that are not tile multiples.  {32,2}:
    N a multiple of 8 (rows and column chunks clamped, partial last K step) and N
    not (the chunk N cuts read by elements).  {32,3}: N a multiple of 4 (rows and
    column groups clamped, with and without a partial last K step) and neither
    (bounded column groups past N, 64-bit addresses).  Entries of the
    edge rows and columns and random ones within the bound, C's padding columns
    untouched."""
    import torch
    M, N, K = shape
    log(f"gemm {case} large edges {shape}")
    k = 2 if case == "bf16" else 3
    if k == 2:
        lda, ldb = K + 2 - K % 2, N + 4 - N % 2   # rows of A and B start 4-byte aligned
    else:
        lda, ldb = _ld(K, 3) + 4, _ld(N, 3) + 4
    ldc = N + 3
    g = np.random.default_rng(M + 3 * N + K)
    A = orc.pack(32, k, g.standard_normal(M * lda).astype(np.float32))
    B = orc.pack(32, k, g.standard_normal(K * ldb).astype(np.float32))
    C = torch.full((M * ldc,), 7.0, dtype=torch.float32, device=dev)
    flyte.gemm((32, k), (32, k), (32, 4), M, N, K, torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev), C=C,
               lda=lda, ldb=ldb, ldc=ldc, flags=flyte.GEMM_ALL_PRODUCTS if case == "four" else 0)
    Ch = C.cpu().numpy().reshape(M, ldc).astype(np.float64)
    assert np.all(Ch[:, N:] == 7.0)
    rows = np.array([0, 1, 255, 256, 4095, 4096, M - 2, M - 1])
    cols = np.array([0, 7, 255, 256, 4095, 4096, N - 2, N - 1])
    gi, gj = np.meshgrid(rows, cols, indexing="ij")
    ii = np.concatenate([gi.reshape(-1), g.integers(0, M, 512)])
    jj = np.concatenate([gj.reshape(-1), g.integers(0, N, 512)])
    ce, cab = orc.gemm_entries((32, k), (32, k), K, A, lda, B, ldb, ii, jj)
    bound = {"bf16": gam(K, U32), "three": 2.0 ** -14 + gam(3 * K, U32) * (1 + 2.0 ** -7) ** 2,
             "four": gam(4 * K, U32) * (1 + 2.0 ** -7) ** 2}[case]
    assert np.all(np.abs(Ch[ii, jj] - ce) <= bound * cab)


def test_gemm_three_product_huge_lda(dev, orc):
    """{32,3} with a leading dimension so large (6M elements, 18 MB per row) that
    byte offsets within a 256-row tile pass 2^32: the bounded instance addresses
    in 64 bits.  Every entry within the 3-product bound."""
    import torch
    M, N, K, lda = 300, 260, 96, 6_000_000
    log(f"gemm three huge lda {M}x{N}x{K} lda={lda}")
    g = np.random.default_rng(91)
    Ac = orc.pack(32, 3, g.standard_normal(M * K).astype(np.float32))
    ldb = _ld(N, 3)
    B = orc.pack(32, 3, g.standard_normal(K * ldb).astype(np.float32))
    Ad = torch.zeros(M * lda * 3, dtype=torch.uint8, device=dev)
    Ad.view(M, lda * 3)[:, :K * 3] = torch.from_numpy(Ac).to(dev).view(M, K * 3)
    C = flyte.gemm((32, 3), (32, 3), (32, 4), M, N, K, Ad, torch.from_numpy(B).to(dev), lda=lda, ldb=ldb)
    Ch = C.cpu().numpy().reshape(M, N).astype(np.float64)
    del Ad
    ii, jj = all_entries(M, N)
    ce, cab = orc.gemm_entries((32, 3), (32, 3), K, Ac, K, B, ldb, ii, jj)
    bound = 2.0 ** -14 + gam(3 * K, U32) * (1 + 2.0 ** -7) ** 2
    assert np.all(np.abs(Ch.reshape(-1) - ce) <= bound * cab)


@pytest.mark.parametrize("kin,kout", [(5, 5), (6, 8), (8, 3), (3, 7)])
@pytest.mark.parametrize("shape", [(300, 520, 333), (129, 1, 17), (1, 130, 250)])
def test_gemm_ragged_f64(dev, orc, kin, kout, shape):
    """The FP64 path at shapes that are not tile multiples: every entry within the
    bound, bytes of C outside the M x N block untouched."""
    import torch
    log(f"gemm ragged f64 {kin}->{kout} {shape}")
    M, N, K = shape
    lda, ldb, ldc = _ld(K, kin) + 4, _ld(N, kin), _ld(N, kout) + 4
    g = np.random.default_rng(kin * 31 + kout + M)
    A = orc.pack(64, kin, g.standard_normal(M * lda))
    B = orc.pack(64, kin, g.standard_normal(K * ldb))
    C = torch.full((M * ldc * kout,), 0x5A, dtype=torch.uint8, device=dev)
    flyte.gemm((64, kin), (64, kin), (64, kout), M, N, K, torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev),
               C=C if kout < 8 else C.view(torch.float64), lda=lda, ldb=ldb, ldc=ldc, flags=flyte.GEMM_FP64)
    Ch = C.cpu().numpy().reshape(M, ldc * kout)
    assert np.all(Ch[:, N * kout:] == 0x5A)
    Cu = orc.unpack(64, kout, np.ascontiguousarray(Ch[:, :N * kout]).reshape(-1))
    ii, jj = all_entries(M, N)
    ce, cab = orc.gemm_entries((64, kin), (64, kin), K, A, lda, B, ldb, ii, jj)
    m = 8 * kout - 12
    bound = gam(K, U64) * cab + 2.0 ** -(m + 1) * (np.abs(ce) + gam(K, U64) * cab)
    assert np.all(np.abs(Cu - ce) <= bound * (1 + 1e-12))


# ---------------------------------------------------------------- binary64 k <= 4 on bfloat16 pieces
def pieces_bound(kin, allp, K, ce, cab, kout):
    P = kin - 1
    n = P * P if allp else {1: 1, 2: 3, 3: 6}[P]
    drop = 0.0 if (allp or P == 1) else (2.0 ** -14 if P == 2 else 2.0 ** -20 * (1 + 2.0 ** -8))
    e = drop + gam(n * K, U32) * (1 + 2.0 ** -7 + 2.0 ** -14) ** 2
    m = 8 * kout - 12
    return e * cab + 2.0 ** -(m + 1) * (np.abs(ce) + e * cab)


@pytest.mark.parametrize("kin", [2, 3, 4])
@pytest.mark.parametrize("allp", [False, True])
@pytest.mark.parametrize("shape", [(256, 256, 128), (300, 264, 133), (384, 256, 64), (300, 260, 96), (129, 256, 20)])
def test_gemm_pieces_all_entries(dev, orc, kin, allp, shape):
    """Rows of A scaled over 2^-300 .. 2^300 and columns of B over 2^-200 .. 2^200
    (each row or column scales as a whole, exactly): every entry within the pieces
    bound, for a native and two packed output formats."""
    import torch
    log(f"gemm pieces k={kin} all={allp} {shape}")
    M, N, K = shape
    lda, ldb = _ld(K, kin), _ld(N, kin)
    g = np.random.default_rng(kin * 100 + M + N)
    Av = g.standard_normal((M, lda)) * np.exp2(np.round(g.uniform(-300, 300, (M, 1))))
    Bv = g.standard_normal((K, ldb)) * np.exp2(np.round(g.uniform(-200, 200, (1, ldb))))
    A, B = orc.pack(64, kin, Av.reshape(-1)), orc.pack(64, kin, Bv.reshape(-1))
    Ad, Bd = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    ii, jj = all_entries(M, N)
    ce, cab = orc.gemm_entries((64, kin), (64, kin), K, A, lda, B, ldb, ii, jj)
    for kout in (8, kin, 5):
        C = flyte.gemm((64, kin), (64, kin), (64, kout), M, N, K, Ad, Bd, lda=lda, ldb=ldb,
                       flags=flyte.GEMM_ALL_PRODUCTS if allp else 0).cpu().numpy()
        Cu = orc.unpack(64, kout, C.view(np.uint8)) if kout < 8 else C
        err = np.abs(Cu.reshape(-1) - ce)
        assert np.all(err <= pieces_bound(kin, allp, K, ce, cab, kout) * (1 + 1e-9)), (kout, np.max(err / cab))


@pytest.mark.parametrize("kin", [2, 3, 4])
def test_gemm_pieces_integer_data_bit_exact(dev, orc, kin):
    """Small integers: every product of pieces and every FP32 partial sum is exact
    (|C| < 2^24), so the packed C must equal the oracle's pack of the exact product
    bit for bit, in every output format and with either product set."""
    import torch
    log(f"gemm pieces integers k={kin}")
    M, N, K = 256, 256, 192
    g = np.random.default_rng(60 + kin)
    lim = 31 if kin == 2 else 64
    Av = g.integers(-lim, lim + 1, (M, K)).astype(np.float64)
    Bv = g.integers(-lim, lim + 1, (K, N)).astype(np.float64)
    exact = Av @ Bv
    A, B = orc.pack(64, kin, Av.reshape(-1)), orc.pack(64, kin, Bv.reshape(-1))
    Ad, Bd = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    for flags in (0, flyte.GEMM_ALL_PRODUCTS):
        for kout in (2, 3, 4, 5, 8):
            C = flyte.gemm((64, kin), (64, kin), (64, kout), M, N, K, Ad, Bd, flags=flags).cpu().numpy()
            want = orc.pack(64, kout, exact.reshape(-1))
            assert np.array_equal(C if kout < 8 else C.view(np.uint8), want), (flags, kout)


@pytest.mark.parametrize("kin", [2, 3, 4])
def test_gemm_pieces_fallback_bands(dev, orc, kin):
    """Rows and columns that cannot be scaled exactly -- an element 2^-60 below its
    row's largest, a binary64 subnormal, an infinity, a NaN -- send every 128 x 128
    tile of their band to the FP64 matrix cores: those tiles equal the FP64 path's
    result bit for bit, the others meet the pieces bound, and the special values
    propagate exactly (infinities stay infinities here)."""
    import torch
    log(f"gemm pieces fallback k={kin}")
    M, N, K = 640, 512, 64
    g = np.random.default_rng(70 + kin)
    Av = g.standard_normal((M, K))
    Bv = g.standard_normal((K, N))
    Av[5, 3] *= 2.0 ** -60          # row band 0 of A: spread above 2^40
    # row band 2: a binary64 subnormal ({64,2} keeps 4 fraction bits, so one near 2^-1022)
    Av[300, 7] = 2e-308 if kin == 2 else 5e-310
    Bv[9, 200] = np.inf             # column band 1 of B: infinity
    Bv[20, 450] = np.nan            # column band 3: NaN
    A, B = orc.pack(64, kin, Av.reshape(-1)), orc.pack(64, kin, Bv.reshape(-1))
    Ad, Bd = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
    C = flyte.gemm((64, kin), (64, kin), (64, 8), M, N, K, Ad, Bd).cpu().numpy().reshape(M, N)
    F = flyte.gemm((64, kin), (64, kin), (64, 8), M, N, K, Ad, Bd, flags=flyte.GEMM_FP64).cpu().numpy().reshape(M, N)
    band_a = np.zeros(M // 128, bool)
    band_a[[0, 2]] = True
    band_b = np.zeros(N // 128, bool)
    band_b[[1, 3]] = True
    fb = band_a[np.arange(M) // 128][:, None] | band_b[np.arange(N) // 128][None, :]
    assert np.array_equal(C[fb].view(np.uint64), F[fb].view(np.uint64))
    ii, jj = all_entries(M, N)
    ce, cab = orc.gemm_entries((64, kin), (64, kin), K, A, K, B, N, ii, jj)
    ce, cab = ce.reshape(M, N), cab.reshape(M, N)
    ok = ~fb
    assert np.all(np.abs(C[ok] - ce[ok]) <= pieces_bound(kin, False, K, ce[ok], cab[ok], 8) * (1 + 1e-9))
    assert np.all(np.isnan(C[np.isnan(ce)]))
    inf = np.isinf(ce)
    assert inf.sum() > 0 and np.array_equal(C[inf], ce[inf])


@pytest.mark.parametrize("k", [2, 3, 4])
def test_gemm_pieces_benchmark_size_sampled(dev, orc, k):
    """M = N = K = 16384, N(0,1) entries packed to {64,k}, C packed to the same k on
    the bfloat16 pieces: sampled entries within the pieces bound."""
    import torch
    log(f"gemm pieces k={k} 16384^3 sampled")
    n = 16384
    g = torch.Generator(device=dev)
    g.manual_seed(workloads.SEED_BASE + 4)
    v = torch.empty(n * n, dtype=torch.float64, device=dev).normal_(generator=g)
    A = flyte.pack((64, k), v)
    v.normal_(generator=g)
    B = flyte.pack((64, k), v)
    del v
    C = flyte.gemm((64, k), (64, k), (64, k), n, n, n, A, B)
    torch.cuda.synchronize()
    Ah, Bh = A.cpu().numpy(), B.cpu().numpy()
    ii, jj, ce, cab = sampled(orc, (64, k), n, Ah, Bh, n, None, n, 5, count=128)
    idx = torch.from_numpy(((ii * n + jj)[:, None] * k + np.arange(k)[None, :]).reshape(-1)).to(dev)
    got = orc.unpack(64, k, C[idx].cpu().numpy())
    assert np.all(np.abs(got - ce) <= pieces_bound(k, False, n, ce, cab, k) * (1 + 1e-9))
    del A, B, C
    torch.cuda.empty_cache()
