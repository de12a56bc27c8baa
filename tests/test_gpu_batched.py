"""GPU parity of the batched persistent GEMV.

* every y of the persistent, graph-launched kernel equals, bit for bit, a
  per-call fb_gemv_config with the tile the plan chose (and the host loop and
  the loop graph give the same bits);
* graph replays after the inputs change pick up the new inputs;
* sampled descriptors meet the summation bound against the exact oracle;
* the plan's autotuner changes tiles only to ones that keep the above true.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from gpu_helpers import device, gamma, log, native_dtype, unit_roundoff
from paper_1601_07789_amd import flyte, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture(scope="module")
def orc():
    return oracle.default()


def make_batch(dev, count, seed, lo, hi, extra=()):
    import torch
    descs = workloads.batched_descs(count, seed, lo=lo, hi=hi) + list(extra)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    items = []
    for d in descs:
        f = (d["base"], d["k"])
        dt = torch.float32 if d["base"] == 32 else torch.float64
        vals = torch.empty(max(1, d["m"] * d["lda"]), dtype=dt, device=dev).uniform_(-1, 1, generator=g)
        A = flyte.pack(f, vals)
        x = torch.empty(max(1, d["n"]), dtype=dt, device=dev).uniform_(-1, 1, generator=g)
        y = torch.full((max(1, d["m"]),), float("nan"), dtype=dt, device=dev)
        items.append(flyte.GemvItem(f, d["m"], d["n"], d["lda"], A, x, y))
    return items


def per_call(items, plan):
    import torch
    outs = []
    for i, it in enumerate(items):
        y = torch.full_like(it.y, float("nan"))
        if it.m:
            flyte.gemv(it.f, it.A, it.m, it.n, it.x, y=y, lda=it.lda, config=plan.config(i))
        outs.append(y)
    return outs


def same_bits(a, b):
    return np.array_equal(a.cpu().numpy().view(np.uint8), b.cpu().numpy().view(np.uint8))


EXTRA = [dict(base=64, k=5, m=1, n=1, lda=4), dict(base=32, k=3, m=3, n=7, lda=8),
         dict(base=64, k=8, m=0, n=5, lda=5), dict(base=64, k=2, m=700, n=1, lda=2),
         dict(base=32, k=2, m=5, n=3000, lda=3000)]


def test_batched_matches_per_call_bitwise(dev, orc):
    import torch
    log("batched vs per-call")
    items = make_batch(dev, 300, workloads.SEED_BASE + 3, 1, 700, EXTRA)
    plan = flyte.BatchedGemv(items)
    ref = per_call(items, plan)
    for replay in range(3):
        for it in items:
            it.y.fill_(float("nan"))
        plan.launch()
        torch.cuda.synchronize()
        for i, it in enumerate(items):
            if it.m:
                assert same_bits(it.y, ref[i]), (replay, i, it.f, it.m, it.n, plan.config(i))
    for mode in ("loop", "loop_graph"):
        for it in items:
            it.y.fill_(float("nan"))
        getattr(plan, mode)()
        torch.cuda.synchronize()
        for i, it in enumerate(items):
            if it.m:
                assert same_bits(it.y, ref[i]), (mode, i)
    # graph replays read the current inputs
    for it in items:
        it.x.mul_(-2.0)
    plan.launch()
    torch.cuda.synchronize()
    for i, it in enumerate(items[:50]):
        if it.m:
            # scaling x by -2 scales every product and partial sum exactly
            assert same_bits(it.y, -2.0 * ref[i]), i
    # sampled descriptors against the exact oracle
    rng = np.random.default_rng(1)
    for i in list(rng.choice(len(items) - len(EXTRA), 12, replace=False)) + list(range(len(items) - len(EXTRA), len(items))):
        it = items[i]
        if not it.m:
            continue
        base, k = it.f
        A = it.A.cpu().numpy()
        xh = it.x.cpu().numpy()
        exact, absrow = orc.gemv_exact(base, k, it.m, it.n, A, it.lda, xh)
        got = it.y.cpu().numpy().astype(np.float64)
        bound = gamma(max(it.n, 1), base) * absrow + unit_roundoff(base) * np.abs(exact)
        assert np.all(np.abs(got - exact) <= bound), (i, it.f, it.m, it.n)
    plan.close()


def test_batched_tuned_plan(dev):
    import torch
    log("batched tuned plan")
    items = make_batch(dev, 120, workloads.SEED_BASE + 33, 16, 1500)
    plan = flyte.BatchedGemv(items)
    plan.tune(reps=3)
    ref = per_call(items, plan)
    plan.launch()
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        assert same_bits(it.y, ref[i]), (i, plan.config(i))
    assert all(plan.config(i) in (11, 12, 9, 10, 33, 32, 21, 7) for i in range(len(items)))
    plan.close()


def test_empty_and_zero_row_batches(dev):
    import torch
    plan = flyte.BatchedGemv([])
    plan.launch()
    plan.close()
    items = make_batch(dev, 0, 1, 1, 2, [dict(base=64, k=6, m=0, n=9, lda=10)])
    plan = flyte.BatchedGemv(items)
    plan.launch()
    torch.cuda.synchronize()
    plan.close()


def test_batched_benchmark_size_sampled(dev, orc):
    """The 4096-GEMV workload the benchmark times (same generator, seeds and input
    construction), tuned and launched as the persistent graph: every y equals the
    per-call fb_gemv_config of its plan tile bit for bit, and 6 rows of each of 24
    sampled descriptors meet the summation bound against the exact oracle."""
    import torch
    log("batched 4096 benchmark workload")
    descs = workloads.batched_descs(4096, workloads.SEED_BASE + 3)
    g = torch.Generator(device=dev)
    g.manual_seed(workloads.SEED_BASE + 3)
    pool = {32: torch.empty(4096 * 4096, dtype=torch.float32, device=dev).uniform_(-1, 1, generator=g),
            64: torch.empty(4096 * 4096, dtype=torch.float64, device=dev).uniform_(-1, 1, generator=g)}
    items = []
    for d in descs:
        f = (d["base"], d["k"])
        src = pool[d["base"]][: d["m"] * d["lda"]]
        A = flyte.pack(f, src)
        x = pool[d["base"]][1000: 1000 + d["n"]].clone()
        y = torch.full((d["m"],), float("nan"), dtype=src.dtype, device=dev)
        items.append(flyte.GemvItem(f, d["m"], d["n"], d["lda"], A, x, y))
    del pool
    plan = flyte.BatchedGemv(items)
    plan.tune(reps=3)
    plan.launch()
    torch.cuda.synchronize()
    ref = per_call(items, plan)
    torch.cuda.synchronize()
    for i, it in enumerate(items):
        assert same_bits(it.y, ref[i]), (i, it.f, it.m, it.n, plan.config(i))
    rng = np.random.default_rng(11)
    for i in rng.choice(len(items), 24, replace=False):
        it = items[i]
        base, k = it.f
        rows = np.unique(np.concatenate([[0, it.m - 1], rng.integers(0, it.m, 4)]))
        rb = torch.from_numpy((rows[:, None] * (it.lda * k) + np.arange(it.lda * k)[None, :]).reshape(-1)).to(dev)
        sub = it.A[rb].cpu().numpy()
        exact, absrow = orc.gemv_exact(base, k, len(rows), it.n, sub, it.lda, it.x.cpu().numpy())
        got = it.y.cpu().numpy()[rows].astype(np.float64)
        bound = gamma(max(it.n, 1), base) * absrow + unit_roundoff(base) * np.abs(exact)
        assert np.all(np.abs(got - exact) <= bound), (i, it.f, it.m, it.n)
    plan.close()
    del items, ref
    torch.cuda.empty_cache()
