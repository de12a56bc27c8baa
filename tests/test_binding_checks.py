"""The Python binding refuses tensors the kernels cannot address safely (no GPU needed).

Each call checks, before the library sees a pointer, that every tensor is in
device memory, contiguous, of the expected element type and large enough for
the bytes the call touches.  Without a GPU the host tensors used here are
refused at the first of those checks, so no device call is made.
"""
from __future__ import annotations

import pytest
import torch

from paper_1601_07789_amd import flyte


def host(n, dtype=torch.uint8):
    return torch.zeros(n, dtype=dtype)


@pytest.mark.parametrize("call", [
    lambda: flyte.pack((64, 5), host(8, torch.float64)),
    lambda: flyte.unpack((64, 5), host(40)),
    lambda: flyte.dot((64, 3), host(30), host(30)),
    lambda: flyte.axpy((64, 3), 2.0, host(30), host(30)),
    lambda: flyte.scale((32, 3), 2.0, host(30)),
    lambda: flyte.nrm2((64, 6), host(60)),
    lambda: flyte.gemv((64, 5), host(4 * 4 * 5), 4, 4, host(4, torch.float64)),
    lambda: flyte.gemv_ex((64, 5), (64, 8), True, host(4 * 4 * 5), 4, 4, host(4, torch.float64)),
    lambda: flyte.dot_packed((64, 5), (64, 3), host(50), host(50)),
    lambda: flyte.gemm((32, 2), (32, 2), (32, 4), 128, 128, 64, host(128 * 64 * 2), host(64 * 128 * 2)),
])
def test_host_tensors_are_refused(call):
    with pytest.raises(ValueError, match="device memory"):
        call()


def test_non_tensor_is_refused():
    with pytest.raises(TypeError):
        flyte.scale((64, 3), 2.0, [0] * 30, n=10)


def test_gemm_leading_dimension_below_row_length():
    with pytest.raises(ValueError, match="leading dimensions"):
        flyte.gemm((32, 2), (32, 2), (32, 4), 128, 128, 64, host(10), host(10), C=host(10, torch.float32), lda=32)


def test_mat_bytes():
    assert flyte._mat_bytes(0, 5, 8, 3) == 0
    assert flyte._mat_bytes(4, 5, 8, 3) == (3 * 8 + 5) * 3
