"""Calls on several streams at once.

The calls that keep partial results in the per-(device, stream) workspace (dot,
magnitude, transposed GEMV, the {32,3} GEMM split) run on two side streams
concurrently, each with its own inputs; every result equals, bit for bit, the
same call made alone on the default stream (the kernels' summation order does
not depend on the stream, and each stream has its own workspace).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_helpers import device, log
from paper_1601_07789_amd import flyte, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


def _inputs(orc, dev, seed):
    import torch
    n = (1 << 20) + 37
    x = orc.pack(64, 5, workloads.uniform(n, seed))
    y = orc.pack(64, 5, workloads.uniform(n, seed + 1))
    m, nn = 3000, 2048
    A = orc.pack(64, 6, workloads.uniform(m * nn, seed + 2))
    xv = workloads.uniform(m, seed + 3)
    M = N = 256
    K = 192
    Ag = orc.pack(32, 3, workloads.normal(M * K, seed + 4))
    Bg = orc.pack(32, 3, workloads.normal(K * N, seed + 5))
    t = lambda a: torch.from_numpy(a).to(dev)
    return dict(x=t(x), y=t(y), A=t(A), xv=t(xv), m=m, n=nn, Ag=t(Ag), Bg=t(Bg), M=M, N=N, K=K)


def _run(d, stream=None):
    dot = flyte.dot((64, 5), d["x"], d["y"], stream=stream)
    nrm = flyte.nrm2((64, 5), d["x"], stream=stream)
    yt = flyte.gemv_ex((64, 6), (64, 8), True, d["A"], d["m"], d["n"], d["xv"], stream=stream)
    C = flyte.gemm((32, 3), (32, 3), (32, 4), d["M"], d["N"], d["K"], d["Ag"], d["Bg"], stream=stream)
    return dot, nrm, yt, C


def test_side_streams_match_default_stream(dev, orc):
    import torch
    log("side streams")
    data = [_inputs(orc, dev, 500 + 10 * i) for i in range(2)]
    ref = []
    for d in data:
        ref.append([r.clone() for r in _run(d)])
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(device=dev) for _ in data]
    for rep in range(3):
        outs = []
        for d, s in zip(data, streams):
            with torch.cuda.stream(s):
                outs.append(_run(d, stream=s))
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, ref)):
            for a, b in zip(o, r):
                assert np.array_equal(a.cpu().numpy().reshape(-1).view(np.uint8),
                                      b.cpu().numpy().reshape(-1).view(np.uint8)), (rep, i)
