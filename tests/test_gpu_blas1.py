"""GPU parity of fb_axpy (bit-exact) and fb_dot (within the summation bound)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_helpers import FORMATS, bits_dtype, device, dot_bound_ok, log, mixed, native_dtype
from paper_1601_07789_amd import flyte, workloads

pytestmark = pytest.mark.gpu

ALPHA = float.fromhex("0x1.5555555555555p-2")   # RN(1/3) in binary64


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


@pytest.mark.parametrize("f", FORMATS)
def test_axpy_bit_exact(dev, orc, f):
    import torch
    base, k = f
    log(f"axpy {f}")
    for n in [1, 3, 4, 5, 17, 1000, (1 << 20) + 3]:
        x = orc.pack(base, k, mixed(base, n, 11 + n))
        y = orc.pack(base, k, mixed(base, n, 12 + n))
        want = orc.axpy(base, k, ALPHA, x, y)
        yd = torch.from_numpy(y.copy()).to(dev)
        flyte.axpy(f, ALPHA, torch.from_numpy(x).to(dev), yd)
        got = yd.cpu().numpy()
        assert np.array_equal(got, want), (n, np.nonzero(got != want)[0][:10])


@pytest.mark.parametrize("k", [3, 4, 5, 6, 7, 8])
def test_axpy_streaming_size_sampled(dev, orc, k):
    """n = 2^28 (the streaming workload), entries U(-1,1) packed; 100k sampled elements."""
    import torch
    log(f"axpy 2^28 sampled k={k}")
    n = 1 << 28
    g = torch.Generator(device=dev)
    g.manual_seed(workloads.SEED_BASE + 1)
    xv = torch.empty(n, dtype=torch.float64, device=dev).uniform_(-1.0, 1.0, generator=g)
    x = flyte.pack((64, k), xv)
    xv.uniform_(-1.0, 1.0, generator=g)
    y = flyte.pack((64, k), xv)
    del xv
    rng = np.random.default_rng(6)
    idx = np.concatenate([np.sort(rng.choice(n, 100_000, replace=False)), [0, n - 1]])
    bidx = torch.from_numpy((idx[:, None] * k + np.arange(k)[None, :]).reshape(-1)).to(dev)
    xs = x[bidx].cpu().numpy()
    ys = y[bidx].cpu().numpy()
    flyte.axpy((64, k), ALPHA, x, y)
    got = y[bidx].cpu().numpy()
    assert np.array_equal(got, orc.axpy(64, k, ALPHA, xs, ys))
    del x, y
    torch.cuda.empty_cache()


@pytest.mark.parametrize("f", FORMATS)
def test_dot_mixed_population(dev, orc, f):
    """With NaN/Inf present the result is NaN; on the finite subset it meets the bound."""
    import torch
    base, k = f
    log(f"dot {f}")
    n = 1 << 20
    xb = mixed(base, n, workloads.SEED_BASE)
    yb = mixed(base, n, workloads.SEED_BASE + 100)
    x, y = orc.pack(base, k, xb), orc.pack(base, k, yb)
    got = flyte.dot(f, torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)).item()
    assert np.isnan(got)
    # finite subset: every special (non-finite, subnormal, and the huge ties and
    # max-finite values whose products overflow) replaced by +0; what stays is
    # the N(0,1) * 2^U part of the population
    big = 2.0 ** 64 if base == 64 else 2.0 ** 34
    def finite(bits):
        v = bits.view(native_dtype(base)).copy()
        lim = np.finfo(native_dtype(base)).tiny
        bad = ~np.isfinite(v) | (np.abs(v) < lim) | (np.abs(v) > big)
        v[bad] = 0
        return v
    xf, yf = orc.pack(base, k, finite(xb)), orc.pack(base, k, finite(yb))
    xd, yd = torch.from_numpy(xf).to(dev), torch.from_numpy(yf).to(dev)
    got = flyte.dot(f, xd, yd).item()
    exact = orc.dot_exact(base, k, xf, yf)
    ax = np.abs(orc.unpack(base, k, xf).astype(np.float64))
    ay = np.abs(orc.unpack(base, k, yf).astype(np.float64))
    absdot = float(np.dot(ax, ay)) * (1 + 1e-12)
    assert dot_bound_ok(got, exact, absdot, n, base), (got, exact)
    again = flyte.dot(f, xd, yd).item()
    assert np.array_equal(np.array(got), np.array(again))   # fixed reduction order


@pytest.mark.parametrize("f", [(32, 3), (64, 3), (64, 5), (64, 8)])
def test_dot_ragged_and_empty(dev, orc, f):
    import torch
    base, k = f
    for n in [0, 1, 2, 3, 5, 7, 9, 31, 1025, 100003]:
        xv = workloads.uniform(n, 3 + n, dtype=native_dtype(base))
        yv = workloads.uniform(n, 4 + n, dtype=native_dtype(base))
        x, y = orc.pack(base, k, xv), orc.pack(base, k, yv)
        got = flyte.dot(f, torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev), n=n).item()
        exact = orc.dot_exact(base, k, x, y)
        absdot = float(np.dot(np.abs(orc.unpack(base, k, x).astype(np.float64)),
                              np.abs(orc.unpack(base, k, y).astype(np.float64)))) * (1 + 1e-12)
        assert dot_bound_ok(got, exact, absdot, max(n, 1), base), (n, got, exact)
