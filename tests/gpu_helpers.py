"""Shared helpers for the GPU parity tests (inputs, bounds, device)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_1601_07789_amd import workloads

FORMATS = workloads.FORMATS


def device():
    torch = pytest.importorskip("torch")
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


def native_dtype(base):
    return np.float32 if base == 32 else np.float64


def bits_dtype(base):
    return np.uint32 if base == 32 else np.uint64


def unit_roundoff(base):
    return 2.0 ** -24 if base == 32 else 2.0 ** -53


def gamma(n, base):
    u = unit_roundoff(base)
    return n * u / (1.0 - n * u)


def mixed(base, n, seed):
    """Mixed special/finite bit patterns of the base type."""
    if base == 64:
        return workloads.mixed_binary64(n, seed)
    return workloads.mixed_binary32(n, seed)


def dot_bound_ok(got, exact, absdot, n, base):
    """|got - exact| <= gamma_n * sum|x_i y_i| + u |exact| (any summation order)."""
    return abs(got - exact) <= gamma(n, base) * absdot + unit_roundoff(base) * abs(exact)


def log(msg):
    print(msg, flush=True)
