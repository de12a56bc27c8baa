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


def test_replay_after_workspace_growth(dev, orc):
    """A graph captured with the stream's small workspace (dot partials) keeps
    working after a later eager call on the same stream grows that workspace
    (a {32,3} GEMM's split planes): the old buffer stays allocated, so each
    replay writes valid memory and returns the captured call's bits."""
    import torch
    log("graph replay after workspace growth")
    t = lambda a: torch.from_numpy(a).to(dev)
    nv = 200003
    u = t(orc.pack(64, 5, workloads.uniform(nv, 710)))
    v = t(orc.pack(64, 5, workloads.uniform(nv, 711)))
    d = torch.empty((), dtype=torch.float64, device=dev)
    s = torch.cuda.Stream(device=dev)      # a fresh stream: its workspace starts small
    with torch.cuda.stream(s):
        flyte.dot((64, 5), u, v, out=d, stream=s)
    torch.cuda.synchronize()
    ref = d.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        flyte.dot((64, 5), u, v, out=d, stream=s)
    torch.cuda.synchronize()
    M = N = K = 512
    A = t(orc.pack(32, 3, workloads.normal(M * K, 712)))
    B = t(orc.pack(32, 3, workloads.normal(K * N, 713)))
    with torch.cuda.stream(s):
        C = flyte.gemm((32, 3), (32, 3), (32, 4), M, N, K, A, B, stream=s)   # grows the workspace
    torch.cuda.synchronize()
    for rep in range(3):
        d.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(d.cpu().numpy().reshape(-1).view(np.uint8), ref.cpu().numpy().reshape(-1).view(np.uint8)), rep
    assert torch.isfinite(C).all().item()
