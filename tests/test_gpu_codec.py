"""GPU parity of fb_pack / fb_unpack against the oracle: bit-exact.

* the mixed special/finite population (2^20 values) for every format;
* every binary32 input for k = 2 and k = 3 (exhaustive);
* ragged lengths and 4-byte-aligned sub-ranges with canary bytes on both sides
  (no write outside the range, tails handled);
* the streaming size (2^28 binary64 values) with sampled checks.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_helpers import FORMATS, bits_dtype, device, log, mixed, native_dtype
from paper_1601_07789_amd import flyte, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


@pytest.mark.parametrize("f", FORMATS)
def test_pack_unpack_mixed_population(dev, orc, f):
    import torch
    base, k = f
    log(f"pack/unpack mixed population {f}")
    bits = mixed(base, 1 << 20, workloads.SEED_BASE)
    want = orc.pack(base, k, bits)
    got = flyte.pack(f, torch.from_numpy(bits.view(native_dtype(base))).to(dev)).cpu().numpy()
    assert np.array_equal(got, want), np.nonzero(got != want)[0][:10]
    un_want = orc.unpack(base, k, want).view(bits_dtype(base))
    un_got = flyte.unpack(f, torch.from_numpy(want).to(dev)).cpu().numpy().view(bits_dtype(base))
    assert np.array_equal(un_got, un_want)
    # idempotence on the device: pack(unpack(pack(x))) == pack(x)
    again = flyte.pack(f, flyte.unpack(f, torch.from_numpy(got).to(dev))).cpu().numpy()
    assert np.array_equal(again, got)


@pytest.mark.parametrize("k", [2, 3])
def test_pack_exhaustive_binary32(dev, orc, k):
    import torch
    from concurrent.futures import ThreadPoolExecutor
    log(f"exhaustive binary32 k={k}")
    chunk = 1 << 26
    pool = ThreadPoolExecutor(8)

    def host(start):
        u = np.arange(start, start + chunk, dtype=np.uint64).astype(np.uint32)
        return orc.pack(32, k, u)

    futs = [pool.submit(host, s) for s in range(0, 1 << 32, chunk)]
    for i, start in enumerate(range(0, 1 << 32, chunk)):
        u = torch.arange(start, start + chunk, dtype=torch.int64, device=dev).to(torch.int32)
        got = flyte.pack((32, k), u.view(torch.float32)).cpu().numpy()
        want = futs[i].result()
        if not np.array_equal(got, want):
            bad = np.nonzero(got != want)[0][:5]
            pytest.fail(f"k={k} chunk {start:#x}: bytes {bad}")
        # and every k-byte pattern in this chunk range unpacks as the oracle does
        if start < (1 << (8 * k)):
            q = np.arange(start, min(start + chunk, 1 << (8 * k)), dtype=np.uint64)
            qb = q.astype(np.uint32).view(np.uint8).reshape(-1, 4)[:, :k].reshape(-1).copy()
            ug = flyte.unpack((32, k), torch.from_numpy(qb).to(dev)).cpu().numpy().view(np.uint32)
            uw = orc.unpack(32, k, qb).view(np.uint32)
            assert np.array_equal(ug, uw)
    pool.shutdown()


LENGTHS = [1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 31, 33, 63, 65, 127, 129, 1023, 1025, 4099, 65537]


@pytest.mark.parametrize("f", FORMATS)
def test_ragged_subranges_with_canaries(dev, orc, f):
    import torch
    base, k = f
    log(f"ragged sub-ranges {f}")
    nd = native_dtype(base)
    for n in LENGTHS:
        vals = mixed(base, max(n, 10), 7 + n)[:n]
        # packed sub-range starts at an element whose byte offset is a multiple of 4
        start_elem = 4 // np.gcd(4, k) * 3
        pad = 64
        total = pad + (start_elem + n) * k + pad
        buf = torch.full((total,), 0xA5, dtype=torch.uint8, device=dev)
        sub = buf[pad + start_elem * k: pad + (start_elem + n) * k]
        flyte.pack(f, torch.from_numpy(vals.view(nd)).to(dev), out=sub, n=n)
        host = buf.cpu().numpy()
        want = orc.pack(base, k, vals)
        assert np.array_equal(host[pad + start_elem * k: pad + (start_elem + n) * k], want), n
        assert np.all(host[:pad + start_elem * k] == 0xA5) and np.all(host[pad + (start_elem + n) * k:] == 0xA5), n
        # unpack into a native sub-range with canaries
        nat = torch.full((n + 8,), -7.0, dtype=torch.float32 if base == 32 else torch.float64, device=dev)
        flyte.unpack(f, sub, n=n, out=nat[4:4 + n])
        h = nat.cpu().numpy()
        assert np.array_equal(h[4:4 + n].view(bits_dtype(base)), orc.unpack(base, k, want).view(bits_dtype(base)))
        assert np.all(h[:4] == -7.0) and np.all(h[4 + n:] == -7.0)


def test_zero_length_is_a_no_op(dev):
    import torch
    buf = torch.full((16,), 0x5A, dtype=torch.uint8, device=dev)
    src = torch.zeros(4, dtype=torch.float64, device=dev)
    flyte.pack((64, 5), src, out=buf, n=0)
    assert torch.all(buf == 0x5A).item()


@pytest.mark.parametrize("k", [3, 5, 8])
def test_pack_streaming_size_sampled(dev, orc, k):
    """2^28 binary64 values (the streaming workload size), 200k sampled positions."""
    import torch
    log(f"pack 2^28 sampled k={k}")
    n = 1 << 28
    g = torch.Generator(device=dev)
    g.manual_seed(workloads.SEED_BASE + 1)
    vals = torch.empty(n, dtype=torch.float64, device=dev).uniform_(-1.0, 1.0, generator=g)
    packed = flyte.pack((64, k), vals)
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(n, 200_000, replace=False))
    idx = np.concatenate([idx, [0, 1, n - 2, n - 1]])
    sv = vals[torch.from_numpy(idx).to(dev)].cpu().numpy()
    want = orc.pack(64, k, sv).reshape(-1, k)
    bidx = torch.from_numpy((idx[:, None] * k + np.arange(k)[None, :]).reshape(-1)).to(dev)
    got = packed[bidx].cpu().numpy().reshape(-1, k)
    assert np.array_equal(got, want)
    un = flyte.unpack((64, k), packed)
    ug = un[torch.from_numpy(idx).to(dev)].cpu().numpy()
    assert np.array_equal(ug.view(np.uint64), orc.unpack(64, k, want.reshape(-1)).view(np.uint64))
    del vals, packed, un
    torch.cuda.empty_cache()
