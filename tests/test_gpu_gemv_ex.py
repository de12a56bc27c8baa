"""GPU parity of the packed-output and transposed GEMV (fb_gemv_ex) and of the
packed dot (fb_dot_packed).

* packed y (trans = 0): bit-identical to the oracle's pack (in y's rounding
  mode) of the native y that fb_gemv computes with the same tile;
* transposed y = A^T x: every column within the summation bound against the
  exact oracle, ragged shapes, padded rows, tails narrower than a unit, the
  8192 x 8192 streaming size (sampled columns); its packed y bit-identical to the
  oracle's pack of its native y;
* packed dot: bit-identical to the oracle's pack of fb_dot's native result.
"""
from __future__ import annotations

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


def outputs_for(base):
    return [(base, k) for k in ((2, 3, 4) if base == 32 else (2, 3, 5, 6, 7, 8))]


@pytest.mark.parametrize("f", FORMATS)
def test_gemv_packed_y_matches_pack_of_native(dev, orc, f):
    import torch
    base, k = f
    G = 4 // np.gcd(4, k)
    m, n = 203, 517
    lda = (n + G - 1) // G * G
    A = orc.pack(base, k, workloads.uniform(m * lda, 81, dtype=native_dtype(base)))
    x = workloads.uniform(n, 82, dtype=native_dtype(base))
    Ad, xd = torch.from_numpy(A).to(dev), torch.from_numpy(x).to(dev)
    y_native = flyte.gemv(f, Ad, m, n, xd, lda=lda).cpu().numpy()
    for fy in outputs_for(base):
        for mode in (0, 1, 2):
            got = flyte.gemv_ex(f, (fy[0], fy[1], mode), False, Ad, m, n, xd, lda=lda).cpu().numpy()
            want = orc.pack(base, fy[1], y_native, mode)
            assert np.array_equal(got.view(np.uint8), want), (fy, mode)


def check_cols(got, exact, abscol, m, base):
    bound = gamma(max(m, 1), base) * abscol + unit_roundoff(base) * np.abs(exact)
    return np.nonzero(~(np.abs(got.astype(np.float64) - exact) <= bound))[0]


@pytest.mark.parametrize("f", FORMATS)
def test_gemv_transposed(dev, orc, f):
    import torch
    base, k = f
    log(f"gemv transposed {f}")
    G = 4 // np.gcd(4, k)
    for m, n in [(1, 1), (3, 7), (17, 1029), (300, 255), (2000, 70), (64, 4099), (700, 2051), (3001, 9)]:
        lda = (n + G - 1) // G * G + G
        A = orc.pack(base, k, workloads.uniform(m * lda, m + n, dtype=native_dtype(base)))
        x = workloads.uniform(m, 3 * m + 1, dtype=native_dtype(base))
        Ad, xd = torch.from_numpy(A).to(dev), torch.from_numpy(x).to(dev)
        y = flyte.gemv_ex(f, f if k * 8 == base else (base, base // 8), True, Ad, m, n, xd, lda=lda).cpu().numpy()
        exact, abscol = orc.gemv_t_exact(base, k, m, n, A, lda, x)
        bad = check_cols(y, exact, abscol, m, base)
        assert bad.size == 0, (m, n, bad[:5])
        for fy in outputs_for(base)[:2]:
            got = flyte.gemv_ex(f, (fy[0], fy[1], 2), True, Ad, m, n, xd, lda=lda).cpu().numpy()
            assert np.array_equal(got.view(np.uint8), orc.pack(base, fy[1], y, 2)), (m, n, fy)


def test_gemv_transposed_empty(dev):
    import torch
    y = torch.full((5,), 3.0, dtype=torch.float64, device=dev)
    A = torch.zeros(40, dtype=torch.uint8, device=dev)
    x = torch.zeros(1, dtype=torch.float64, device=dev)
    flyte.gemv_ex((64, 8), (64, 8), True, A, 0, 5, x, y=y, lda=5)     # m = 0: y = 0
    assert torch.all(y == 0).item()
    flyte.gemv_ex((64, 8), (64, 8), True, A, 3, 0, x, y=y, lda=0)     # n = 0: nothing


@pytest.mark.parametrize("k", [3, 4, 5, 7, 8])
def test_gemv_transposed_streaming_size_sampled(dev, orc, k):
    import torch
    log(f"gemv transposed 8192^2 k={k}")
    m = n = 8192
    g = torch.Generator(device=dev)
    g.manual_seed(workloads.SEED_BASE + 1)
    vals = torch.empty(m * n, dtype=torch.float64, device=dev).uniform_(-1.0, 1.0, generator=g)
    A = flyte.pack((64, k), vals)
    del vals
    x = torch.from_numpy(workloads.uniform(m, workloads.SEED_BASE + 102)).to(dev)
    y = flyte.gemv_ex((64, k), (64, 8), True, A, m, n, x).cpu().numpy()
    cols = np.concatenate([[0, n - 1], np.random.default_rng(8).choice(n, 30, replace=False)])
    # gather the sampled columns of A into a small m x len(cols) packed matrix
    idx = torch.from_numpy((np.arange(m)[:, None, None] * (n * k) + cols[None, :, None] * k
                            + np.arange(k)[None, None, :]).reshape(-1)).to(dev)
    sub = A[idx].cpu().numpy()
    exact, abscol = orc.gemv_t_exact(64, k, m, len(cols), sub, len(cols), x.cpu().numpy())
    assert check_cols(y[cols], exact, abscol, m, 64).size == 0
    del A
    torch.cuda.empty_cache()


@pytest.mark.parametrize("f", [(32, 3), (64, 3), (64, 6)])
def test_dot_packed_matches_pack_of_native(dev, orc, f):
    import torch
    base, k = f
    for n in [0, 1, 1000, 1 << 20]:
        x = orc.pack(base, k, workloads.uniform(n, 90 + n, dtype=native_dtype(base)))
        y = orc.pack(base, k, workloads.uniform(n, 91 + n, dtype=native_dtype(base)))
        xd, yd = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
        native = flyte.dot(f, xd, yd, n=n).cpu().numpy().reshape(1)
        for kr in ((2, 3) if base == 32 else (2, 5, 7)):
            for mode in (0, 1, 2):
                got = flyte.dot_packed(f, (base, kr, mode), xd, yd, n=n).cpu().numpy()
                assert np.array_equal(got, orc.pack(base, kr, native, mode)), (n, kr, mode)
