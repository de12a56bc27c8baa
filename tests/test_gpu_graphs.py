"""Calls captured into a graph.

GEMV, dot, the transposed GEMV and axpy are captured on a side stream (after one
eager call of each there, so the stream's workspace exists) and the graph is
replayed several times, with eager work and synchronisation between replays;
every replay equals the eager results bit for bit.
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


def test_capture_and_replay(dev, orc):
    import torch
    log("graph capture")
    t = lambda a: torch.from_numpy(a).to(dev)
    m, n = 1500, 2052
    A = t(orc.pack(64, 5, workloads.uniform(m * n, 700)))
    x = t(workloads.uniform(n, 701))
    xt = t(workloads.uniform(m, 702))
    nv = 100003
    u = t(orc.pack(64, 3, workloads.uniform(nv, 703)))
    v0 = orc.pack(64, 3, workloads.uniform(nv, 704))
    y = torch.empty(m, dtype=torch.float64, device=dev)
    yt = torch.empty(n, dtype=torch.float64, device=dev)
    d = torch.empty((), dtype=torch.float64, device=dev)
    v = t(v0.copy())

    def calls(s):
        flyte.gemv((64, 5), A, m, n, x, y=y, stream=s)
        flyte.gemv_ex((64, 5), (64, 8), True, A, m, n, xt, y=yt, stream=s)
        flyte.dot((64, 3), u, v, out=d, stream=s)
        flyte.axpy((64, 3), 0.5, u, v, stream=s)

    s = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(s):
        calls(s)                                   # eager, on the capture stream
    torch.cuda.synchronize()
    ref = [y.clone(), yt.clone(), d.clone(), v.clone()]
    g = torch.cuda.CUDAGraph()
    v.copy_(t(v0))
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        calls(s)
    torch.cuda.synchronize()
    for rep in range(4):
        y.zero_(); yt.zero_(); d.zero_()
        v.copy_(t(v0))                             # axpy updates v in place
        junk = torch.ones(1 << 20, device=dev).sum()   # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert junk.item() == float(1 << 20)
        for a, b in zip([y, yt, d, v], ref):
            assert np.array_equal(a.cpu().numpy().reshape(-1).view(np.uint8),
                                  b.cpu().numpy().reshape(-1).view(np.uint8)), rep
