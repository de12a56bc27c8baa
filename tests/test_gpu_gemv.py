"""GPU parity of fb_gemv against the exact oracle (bound per row), every tile
configuration, ragged shapes, padded leading dimensions, and the 8192 x 8192
streaming workload (sampled rows) in the launch configuration the benchmark
uses."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import oracle
from gpu_helpers import FORMATS, device, gamma, log, native_dtype, unit_roundoff
from paper_1601_07789_amd import flyte, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


def check_rows(got, exact, absrow, n, base):
    bound = gamma(max(n, 1), base) * absrow + unit_roundoff(base) * np.abs(exact)
    bad = np.nonzero(~(np.abs(got.astype(np.float64) - exact) <= bound))[0]
    return bad


@pytest.mark.parametrize("f", FORMATS)
def test_gemv_every_config(dev, orc, f):
    import torch
    base, k = f
    log(f"gemv configs {f}")
    G = 4 // np.gcd(4, k)
    m, n = 131, 1029
    lda = (n + G - 1) // G * G + 3 * G     # padded rows, still 4-byte aligned
    vals = workloads.uniform(m * lda, 21, dtype=native_dtype(base))
    A = orc.pack(base, k, vals)
    x = workloads.uniform(n, 22, dtype=native_dtype(base))
    exact, absrow = orc.gemv_exact(base, k, m, n, A, lda, x)
    Ad, xd = torch.from_numpy(A).to(dev), torch.from_numpy(x).to(dev)
    for cfg in range(flyte.gemv_num_configs()):
        y = torch.full((m + 4,), 99.0, dtype=torch.float32 if base == 32 else torch.float64, device=dev)
        flyte.gemv(f, Ad, m, n, xd, y=y[:m], lda=lda, config=cfg)
        yh = y.cpu().numpy()
        bad = check_rows(yh[:m], exact, absrow, n, base)
        assert bad.size == 0, (cfg, bad[:5], yh[bad[:5]], exact[bad[:5]])
        assert np.all(yh[m:] == 99.0), cfg
        y2 = flyte.gemv(f, Ad, m, n, xd, lda=lda, config=cfg).cpu().numpy()
        assert np.array_equal(y2.view(np.uint8), yh[:m].view(np.uint8)), cfg   # deterministic


SHAPES = [(1, 1), (1, 7), (3, 1), (5, 3), (64, 64), (65, 63), (7, 4099), (300, 17), (1000, 130)]


@pytest.mark.parametrize("f", [(32, 2), (32, 3), (64, 2), (64, 3), (64, 5), (64, 6), (64, 7), (64, 8)])
def test_gemv_small_and_ragged_shapes(dev, orc, f):
    import torch
    base, k = f
    G = 4 // np.gcd(4, k)
    for m, n in SHAPES:
        lda = (n + G - 1) // G * G
        A = orc.pack(base, k, workloads.uniform(m * lda, m + n, dtype=native_dtype(base)))
        x = workloads.uniform(n, 2 * n, dtype=native_dtype(base))
        exact, absrow = orc.gemv_exact(base, k, m, n, A, lda, x)
        Ad, xd = torch.from_numpy(A).to(dev), torch.from_numpy(x).to(dev)
        y = flyte.gemv(f, Ad, m, n, xd, lda=lda).cpu().numpy()
        assert check_rows(y, exact, absrow, n, base).size == 0, (m, n)


def test_gemv_empty(dev):
    import torch
    y = torch.full((4,), 5.0, dtype=torch.float64, device=dev)
    A = torch.zeros(8, dtype=torch.uint8, device=dev)
    x = torch.zeros(4, dtype=torch.float64, device=dev)
    flyte.gemv((64, 5), A, 0, 4, x, y=y)
    flyte.gemv((64, 5), A, 4, 0, x, y=y)   # n = 0: y = 0
    assert torch.all(y == 0).item()


TILE_CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1601_07789_amd",
                          "tuned", "gemv_mi355x.json")


@pytest.fixture()
def bench_tiles():
    """The committed tile cache that the benchmark loads, for the length of a test."""
    flyte.tune_load(TILE_CACHE)
    with open(TILE_CACHE) as fh:
        entries = json.load(fh)["entries"]
    yield {(e["base"], e["k"]): e["tile"] for e in entries}
    flyte.tune_clear()


@pytest.mark.parametrize("k", [3, 4, 5, 6, 7, 8])
def test_gemv_streaming_size_sampled(dev, orc, bench_tiles, k):
    """A 8192 x 8192 (binary64-derived k bytes, U(-1,1)), x U(-1,1): 48 sampled rows,
    with the tile the benchmark runs (the committed cache)."""
    import torch
    log(f"gemv 8192^2 k={k}")
    m = n = 8192
    assert flyte.tune_lookup((64, k), m, n) == bench_tiles[(64, k)]
    g = torch.Generator(device=dev)
    g.manual_seed(workloads.SEED_BASE + 1)
    vals = torch.empty(m * n, dtype=torch.float64, device=dev).uniform_(-1.0, 1.0, generator=g)
    A = flyte.pack((64, k), vals)
    del vals
    x = torch.from_numpy(workloads.uniform(n, workloads.SEED_BASE + 101)).to(dev)
    y = flyte.gemv((64, k), A, m, n, x).cpu().numpy()
    rows = np.concatenate([[0, 1, m - 1], np.random.default_rng(7).choice(m, 45, replace=False)])
    rb = torch.from_numpy((rows[:, None] * (n * k) + np.arange(n * k)[None, :]).reshape(-1)).to(dev)
    Ah = A[rb].cpu().numpy()
    exact, absrow = orc.gemv_exact(64, k, len(rows), n, Ah, n, x.cpu().numpy())
    assert check_rows(y[rows], exact, absrow, n, 64).size == 0
    del A
    torch.cuda.empty_cache()


@pytest.mark.parametrize("f", [(64, 5), (32, 3)])
def test_tune_gemv_records_a_valid_choice(dev, orc, f):
    """fb_tune_gemv times every tile on the caller's buffers, records the fastest for the
    shape bucket and returns it; fb_gemv then uses it, bit-identical to that forced tile,
    and within the bound against the exact oracle."""
    import torch
    base, k = f
    log(f"tune gemv {f}")
    m, n = 1536, 2052
    A = orc.pack(base, k, workloads.uniform(m * n, 31, dtype=native_dtype(base)))
    x = workloads.uniform(n, 32, dtype=native_dtype(base))
    Ad, xd = torch.from_numpy(A).to(dev), torch.from_numpy(x).to(dev)
    flyte.tune_clear()
    try:
        y = torch.empty(m, dtype=torch.float32 if base == 32 else torch.float64, device=dev)
        best = flyte.tune_gemv(f, Ad, m, n, xd, y, reps=2)
        assert 0 <= best < flyte.gemv_num_configs()
        assert flyte.tune_lookup(f, m, n) == best
        auto = flyte.gemv(f, Ad, m, n, xd).cpu().numpy()
        forced = flyte.gemv(f, Ad, m, n, xd, config=best).cpu().numpy()
        assert np.array_equal(auto.view(np.uint8), forced.view(np.uint8))
        exact, absrow = orc.gemv_exact(base, k, m, n, A, n, x)
        assert check_rows(auto, exact, absrow, n, base).size == 0
    finally:
        flyte.tune_clear()
