"""GPU test of the allocation-free entry point fb_dot_noalloc, called through
the C ABI: its result must equal fb_dot's bit for bit (same kernels, same
order), on two calls in a row with the second on a smaller input, for binary32
and binary64 formats, including the byte tail of a ragged length."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from gpu_helpers import device, log
from paper_1601_07789_amd import flyte, workloads

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("f", [(64, 5), (64, 8), (32, 3), (64, 2)])
def test_dot_noalloc_matches_dot(f):
    import torch
    dev = device()
    lib = flyte.load()
    base, k = f
    nd = np.float32 if base == 32 else np.float64
    td = torch.float32 if base == 32 else torch.float64
    for n in (3_000_017, 70_001):          # second call smaller; both ragged
        log(f"dot_noalloc {f} n={n}")
        xv = torch.from_numpy(workloads.uniform(n, 11, dtype=nd)).to(dev)
        yv = torch.from_numpy(workloads.uniform(n, 12, dtype=nd)).to(dev)
        x, y = flyte.pack(f, xv), flyte.pack(f, yv)
        ref = torch.full((1,), float("nan"), dtype=td, device=dev)
        got = torch.full((1,), float("nan"), dtype=td, device=dev)
        stream = torch.cuda.current_stream().cuda_stream
        fm = flyte.fmt(f)
        assert lib.fb_dot(fm, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                          ctypes.c_void_p(ref.data_ptr()), ctypes.c_void_p(stream)) == flyte.FB_OK
        assert lib.fb_dot_noalloc(fm, n, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                  ctypes.c_void_p(got.data_ptr()), ctypes.c_void_p(stream)) == flyte.FB_OK
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy().view(np.uint8), ref.cpu().numpy().view(np.uint8)), (f, n)
        assert np.isfinite(got.cpu().numpy()).all()
