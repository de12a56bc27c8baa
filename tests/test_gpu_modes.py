"""GPU parity of the other rounding modes (toward zero, to odd), scale and magnitude.

* fb_pack in every mode, bit-exact against the oracle: the mixed population for
  every format, and every binary32 input for {32,2} rounding to odd;
* fb_axpy and fb_scale in every mode, bit-exact, ragged lengths;
* fb_gemm (FP64, packed C) in every mode: integer data, exact in FP64, so C must
  equal the oracle's pack of the exact product in that mode;
* fb_nrm2 within its bound against the exact norm.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_helpers import FORMATS, bits_dtype, device, gamma, log, mixed, native_dtype, unit_roundoff
from paper_1601_07789_amd import flyte, workloads

pytestmark = pytest.mark.gpu
ALPHA = float.fromhex("0x1.5555555555555p-2")


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


@pytest.mark.parametrize("f", FORMATS)
@pytest.mark.parametrize("mode", [1, 2])
def test_pack_modes_mixed_population(dev, orc, f, mode):
    import torch
    base, k = f
    bits = mixed(base, 1 << 18, workloads.SEED_BASE + mode)
    want = orc.pack(base, k, bits, mode)
    got = flyte.pack((base, k, mode), torch.from_numpy(bits.view(native_dtype(base))).to(dev)).cpu().numpy()
    assert np.array_equal(got, want), np.nonzero(got != want)[0][:8]


def test_pack_to_odd_exhaustive_binary32_k2(dev, orc):
    import torch
    from concurrent.futures import ThreadPoolExecutor
    log("exhaustive binary32 k=2 to odd")
    chunk = 1 << 26
    pool = ThreadPoolExecutor(8)
    futs = {s: pool.submit(lambda s=s: orc.pack(32, 2, np.arange(s, s + chunk, dtype=np.uint64).astype(np.uint32), 2))
            for s in range(0, 1 << 32, chunk)}
    for s in range(0, 1 << 32, chunk):
        u = torch.arange(s, s + chunk, dtype=torch.int64, device=dev).to(torch.int32)
        got = flyte.pack((32, 2, 2), u.view(torch.float32)).cpu().numpy()
        assert np.array_equal(got, futs[s].result()), hex(s)
    pool.shutdown()


@pytest.mark.parametrize("f", [(32, 2), (32, 3), (64, 2), (64, 3), (64, 5), (64, 6), (64, 7)])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_axpy_and_scale_modes(dev, orc, f, mode):
    import torch
    base, k = f
    for n in [1, 5, 1003, (1 << 16) + 7]:
        x = orc.pack(base, k, mixed(base, n, 3 + n))
        y = orc.pack(base, k, mixed(base, n, 4 + n))
        yd = torch.from_numpy(y.copy()).to(dev)
        flyte.axpy((base, k, mode), ALPHA, torch.from_numpy(x).to(dev), yd)
        assert np.array_equal(yd.cpu().numpy(), orc.axpy(base, k, ALPHA, x, y, mode)), ("axpy", n)
        xd = torch.from_numpy(x.copy()).to(dev)
        flyte.scale((base, k, mode), ALPHA, xd)
        assert np.array_equal(xd.cpu().numpy(), orc.scale(base, k, ALPHA, x, mode)), ("scale", n)


@pytest.mark.parametrize("mode", [1, 2])
def test_gemm_f64_packed_c_modes_integer_data(dev, orc, mode):
    import torch
    M, N, K = 256, 128, 64
    g = np.random.default_rng(9)
    Av = g.integers(-64, 65, (M, K)).astype(np.float64)
    Bv = g.integers(-64, 65, (K, N)).astype(np.float64)
    exact = Av @ Bv
    for kin in (5, 6):
        A, B = orc.pack(64, kin, Av.reshape(-1)), orc.pack(64, kin, Bv.reshape(-1))
        for kout in (2, 3, 4, 7):
            C = flyte.gemm((64, kin), (64, kin), (64, kout, mode), M, N, K,
                           torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)).cpu().numpy()
            assert np.array_equal(C, orc.pack(64, kout, exact.reshape(-1), mode)), (kin, kout, mode)


@pytest.mark.parametrize("f", [(32, 2), (32, 3), (64, 3), (64, 5), (64, 8)])
def test_nrm2_bound(dev, orc, f):
    import torch
    base, k = f
    for n in [0, 1, 7, 1000, (1 << 20) + 3]:
        x = orc.pack(base, k, workloads.uniform(n, 70 + n, dtype=native_dtype(base)))
        got = flyte.nrm2(f, torch.from_numpy(x).to(dev), n=n).item()
        want = orc.nrm2_exact(base, k, x)
        u = unit_roundoff(base)
        assert abs(got - want) <= (gamma(max(n, 1), base) / 2 + 2 * u) * want, (n, got, want)
