#!/usr/bin/env python3
"""Benchmark of the k-byte GEMV hot path on one MI355X.

Workload: y = A x with A 8192 x 8192 row-major, stored in the binary64-derived
k-byte formats k = 3..8 (entries U(-1,1) packed on the device by fb_pack), x
and y FP64, FP64 accumulation.  One step runs, for every k, one GEMV over each
of R rotating copies of A (R * size(A) >= 1 GiB, so the 256 MB last-level
cache holds none of the A being read).  k = 8 is the FP64-stored baseline; the
vendor FP64 GEMV (torch.mv -> rocBLAS) is timed beside it.

value = algorithmic bytes of every GEMV in the timed region / wall time.
Per-k kernel durations come from HIP events on the launch stream; the
roofline entry reports the GEMV kernels' algorithmic bandwidth against the
8 TB/s HBM peak, with the HBM traffic measured by the committed counter
profile when it matches the kernels and tiles in use.  After the timed region
(reported under "detail"): the transposed GEMV, the codec and BLAS-1 kernels
at 2^28 elements, the batched workload (4096 mixed GEMVs), and the GEMMs (BF16,
3- and 4-product, FP64 with a k-byte C) with the vendor library's GEMMs beside
them; cpu_baseline times the oracle's GEMV on the host.  detail.provenance names
the input seeds, the git commit (when the tree is a repository) and a hash of
the kernel sources.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                       [--no-gemm] [--no-batched] [--no-blas1] [--retune] [--tune-cache PATH]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "k-byte GEMV eff. GB/s (% HBM peak), speedup vs FP64-stored; GEMM TFLOP/s @tol"
DEFAULT_TILES = os.path.join(ROOT, "paper_1601_07789_amd", "tuned", "gemv_mi355x.json")
COUNTERS = os.path.join(ROOT, "profiles", "gemv_8192x8192_k3-8_hbm_counters.md")
HBM_PEAK_GBPS = 8000.0
M = N = 8192
KS = [3, 4, 5, 6, 7, 8]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gemv_bytes(k: int) -> int:
    # A (m*n*k) + x (n*8) + y (m*8)
    return M * N * k + N * 8 + M * 8


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rotate", type=int, default=0, help="A copies per k (0: enough for >= 1 GiB)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gemm", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-blas1", action="store_true")
    ap.add_argument("--retune", action="store_true",
                    help="tune the GEMV tiles with rotating buffers instead of loading the committed cache")
    ap.add_argument("--tune-cache", default=DEFAULT_TILES,
                    help="tile cache to load (default: the committed MI355X cache); with --retune, where to save")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1).", file=sys.stderr)
        return 2

    prov = provenance()      # before the device is touched (it may start git as a child)

    import numpy as np
    import torch

    from paper_1601_07789_amd import flyte, workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    flyte.load()
    stream = torch.cuda.current_stream()

    # ------------------------------------------------------------ inputs
    log("generating inputs")
    g = torch.Generator(device=dev)
    g.manual_seed(workloads.SEED_BASE + 1)
    vals = torch.empty(M * N, dtype=torch.float64, device=dev).uniform_(-1.0, 1.0, generator=g)
    A = {}
    R = {}
    for k in KS:
        R[k] = args.rotate or max(4, -(-(1 << 30) // (M * N * k)))
        first = flyte.pack((64, k), vals)
        A[k] = [first] + [first.clone() for _ in range(R[k] - 1)]
    x = torch.from_numpy(workloads.uniform(N, workloads.SEED_BASE + 101)).to(dev)
    y = torch.empty(M, dtype=torch.float64, device=dev)
    A64 = [vals.view(M, N)] + [vals.view(M, N).clone() for _ in range(R[8] - 1)]
    torch.cuda.synchronize()

    def ev():
        return torch.cuda.Event(enable_timing=True)

    # ------------------------------------------------------------ tile choice (rotating buffers)
    tiles = {}
    if not args.retune and os.path.exists(args.tune_cache):
        flyte.tune_load(args.tune_cache)
        log(f"tiles loaded from {args.tune_cache}")
    if args.retune:
        log("tuning GEMV tiles with rotating buffers")
        for k in KS:
            best = None
            for c in range(flyte.gemv_num_configs()):
                for r in range(R[k]):
                    flyte.gemv((64, k), A[k][r], M, N, x, y=y, config=c)
                e0, e1 = ev(), ev()
                e0.record(stream)
                for rep in range(2):
                    for r in range(R[k]):
                        flyte.gemv((64, k), A[k][r], M, N, x, y=y, config=c)
                e1.record(stream)
                e1.synchronize()
                us = 1000.0 * e0.elapsed_time(e1) / (2 * R[k])
                if best is None or us < best[1]:
                    best = (c, us)
            flyte.tune_record((64, k), M, N, best[0], best[1])
            tiles[k] = best[0]
    for k in KS:
        tiles.setdefault(k, flyte.tune_lookup((64, k), M, N))
    if args.retune and args.tune_cache != DEFAULT_TILES:
        flyte.tune_save(args.tune_cache)

    # ------------------------------------------------------------ timed GEMV sweep
    def step(events=None):
        for k in KS:
            if events is not None:
                events[k][0].record(stream)
            for r in range(R[k]):
                flyte.gemv((64, k), A[k][r], M, N, x, y=y)
            if events is not None:
                events[k][1].record(stream)

    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    per_k_ms = {k: [] for k in KS}
    step_events = [{k: (ev(), ev()) for k in KS} for _ in range(args.steps)]
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(step_events[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for s in range(args.steps):
        for k in KS:
            e0, e1 = step_events[s][k]
            per_k_ms[k].append(e0.elapsed_time(e1) / R[k])
    bytes_per_step = sum(R[k] * gemv_bytes(k) for k in KS)
    ms_per_step = 1000.0 * wall / args.steps
    value = bytes_per_step / (wall / args.steps) / 1e9

    per_k = {}
    for k in KS:
        us = 1000.0 * float(np.mean(per_k_ms[k]))
        gbs = gemv_bytes(k) / (us * 1e-6) / 1e9
        per_k[k] = {"us": round(us, 2), "GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBPS, 4),
                    "tile": tiles[k]}

    # ------------------------------------------------------------ vendor FP64 GEMV (rocBLAS via torch.mv)
    log("timing vendor FP64 GEMV")
    for r in range(len(A64)):
        torch.mv(A64[r], x, out=y)
    e0, e1 = ev(), ev()
    reps = 5
    e0.record(stream)
    for _ in range(reps):
        for r in range(len(A64)):
            torch.mv(A64[r], x, out=y)
    e1.record(stream)
    e1.synchronize()
    vendor_us = 1000.0 * e0.elapsed_time(e1) / (reps * len(A64))
    fp64_stored_us = min(vendor_us, per_k[8]["us"])
    for k in KS:
        per_k[k]["speedup_vs_fp64_stored"] = round(fp64_stored_us / per_k[k]["us"], 3)
        per_k[k]["ideal_8_over_k"] = round(8.0 / k, 3)

    # the transposed GEMV (y = A^T x) on the same matrices
    trans = {}
    for k in KS:
        yt = torch.empty(N, dtype=torch.float64, device=dev)
        for r in range(R[k]):
            flyte.gemv_ex((64, k), (64, 8), True, A[k][r], M, N, x, y=yt)
        e0, e1 = ev(), ev()
        e0.record(stream)
        for r in range(R[k]):
            flyte.gemv_ex((64, k), (64, 8), True, A[k][r], M, N, x, y=yt)
        e1.record(stream)
        e1.synchronize()
        us = 1000.0 * e0.elapsed_time(e1) / R[k]
        trans[k] = {"us": round(us, 2), "GBps": round(gemv_bytes(k) / (us * 1e-6) / 1e9, 1)}

    # roofline over the GEMV launches (one kernel template, six formats)
    tot_bytes = sum(gemv_bytes(k) for k in KS)
    tot_us = sum(per_k[k]["us"] for k in KS)
    achieved = tot_bytes / (tot_us * 1e-6) / 1e9
    traffic = measured_traffic(tiles)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": "flyte::k_gemv (binary64-derived k=3..8, one launch per k; "
                          "achieved = sum of algorithmic bytes / sum of mean launch durations)"}
    del A64

    # ------------------------------------------------------------ measured stream references
    stream_ref = measure_streams(torch, dev, stream)

    # ------------------------------------------------------------ CPU baseline: the oracle
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(A, x, np)

    # ------------------------------------------------------------ GEMM (after the timed region)
    detail = {"per_k": per_k, "transposed_per_k": trans, "vendor_fp64_gemv_us": round(vendor_us, 2), "rotate": R,
              "bytes_per_step": bytes_per_step, "stream_reference": stream_ref,
              "gemv_frac_of_measured_read_stream": round(achieved / stream_ref["read_GBps"], 4)}
    del A
    torch.cuda.empty_cache()
    if not args.no_gemm:
        try:
            detail["gemm"] = bench_gemm(flyte, workloads, torch, np, dev, stream)
        except Exception as e:   # reported, not hidden: the GEMV line stands on its own
            detail["gemm"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_blas1:
        try:
            detail["blas1"] = bench_blas1(flyte, workloads, torch, dev, stream)
        except Exception as e:
            detail["blas1"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_batched:
        try:
            detail["batched"] = bench_batched(flyte, workloads, torch, dev, stream)
        except Exception as e:
            detail["batched"] = {"error": f"{type(e).__name__}: {e}"}

    prov["seeds"] = {"gemv_A": workloads.SEED_BASE + 1, "gemv_x": workloads.SEED_BASE + 101,
                     "gemm_b32": workloads.SEED_BASE + 2, "batched": workloads.SEED_BASE + 3,
                     "gemm_f64": workloads.SEED_BASE + 4, "blas1": workloads.SEED_BASE + 1}
    detail["provenance"] = prov

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "GEMV y=Ax, A 8192x8192 binary64-derived k-byte (k=3..8, U(-1,1)), "
                               "x,y FP64; R rotating A copies per k (>= 1 GiB), one GEMV per copy per step",
                   "m": M, "n": N, "k": KS, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(line), flush=True)
    return 0


def provenance() -> dict:
    """The git commit of the tree (None where the tree carries no repository) and a
    sha256 prefix over the kernel sources and the C header, so a result line names
    the code it measured."""
    import hashlib
    import subprocess
    commit = None
    try:
        r = subprocess.run(["git", "rev-parse", "--show-toplevel", "HEAD"], cwd=ROOT, capture_output=True,
                           text=True, timeout=20)
        out = r.stdout.split()
        # only this tree's own repository (a parent directory's would name other code)
        if r.returncode == 0 and len(out) == 2 and os.path.realpath(out[0]) == os.path.realpath(ROOT):
            commit = out[1]
    except (OSError, subprocess.SubprocessError):
        pass
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1601_07789_amd", "csrc")
    for f in sorted(os.listdir(csrc)) + ["../../include/flyte.h"]:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return {"git_commit": commit, "sources_sha256": h.hexdigest()[:16]}


def source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ["codec.hpp", "gemv_impl.hpp", "gemv.hip"]:
        with open(os.path.join(ROOT, "paper_1601_07789_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(tiles):
    """HBM bytes of one GEMV launch per k, summed over k (the unit of 'achieved'),
    from the committed rocprofv3 counter summary -- or None if the kernel sources
    or the tiles in use differ from those the counters were taken with."""
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None
    if f"source-sha256: {source_hash()}" not in text:
        return None
    rows = {}
    for line in text.splitlines():
        parts = line.split()
        if len(parts) == 4 and parts[0] == "traffic":
            rows[int(parts[1])] = (int(parts[2]), int(parts[3]))
    if any(k not in rows or rows[k][0] != tiles[k] for k in KS):
        return None
    return sum(rows[k][1] for k in KS)


def measure_streams(torch, dev, stream):
    """Plain read and copy bandwidth of the device (vendor kernels: torch.sum and
    copy_ over 4 GiB), as a measured reference next to the nominal 8 TB/s."""
    n = (4 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    out = {}
    for name, fn, nbytes in [("read_GBps", lambda: a.sum(), 8 * n),
                             ("copy_GBps", lambda: b.copy_(a), 16 * n)]:
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(5):
            fn()
        e1.record(stream)
        e1.synchronize()
        out[name] = round(nbytes / (e0.elapsed_time(e1) / 5 * 1e-3) / 1e9, 1)
    del a, b
    torch.cuda.empty_cache()
    return out


def cpu_baseline(A, x, np):
    """The oracle's naive GEMV (sequential fma per row, one thread) on a bounded
    sample of the same workload: the full 8192 x 8192 matrix of each k, passed
    repeatedly until about 2 s of CPU time per k (about 12 s in all)."""
    import oracle
    orc = oracle.default()
    xh = x.cpu().numpy()
    total_bytes, total_s, passes = 0, 0.0, {}
    for k in KS:
        Ah = A[k][0].cpu().numpy()
        p, spent = 0, 0.0
        while spent < 2.0:
            t0 = time.perf_counter()
            orc.gemv_naive(64, k, M, N, Ah, N, xh)
            spent += time.perf_counter() - t0
            p += 1
        total_bytes += p * gemv_bytes(k)
        total_s += spent
        passes[k] = p
    gbs = total_bytes / total_s / 1e9
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle fbo_gemv_naive (one thread), full 8192x8192 GEMV per k = 3..8, "
                      f"passes per k = {passes}; {total_s:.1f} s of CPU time",
            "host": host_cpu()}


def host_cpu():
    """CPU model and logical CPU count of the host the baseline ran on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "available": avail}


def bench_blas1(flyte, workloads, torch, dev, stream):
    """Streaming codec and BLAS-1 kernels on n = 2^28 elements (the 2 GiB FP64 side
    and every packed array exceed the 256 MB last-level cache): algorithmic GB/s and
    fraction of 8 TB/s.  pack: n(W+k) bytes, unpack: n(k+W), axpy: 3nk, dot: 2nk,
    scale (in place): 2nk, nrm2: nk."""
    n = 1 << 28
    g = torch.Generator(device=dev)
    g.manual_seed(workloads.SEED_BASE + 1)
    nat = torch.empty(n, dtype=torch.float64, device=dev).uniform_(-1.0, 1.0, generator=g)
    out = {"n": n}

    def timed(fn, reps=3, warm=3):
        # untimed calls first (the GPU may have idled during the host-side steps before)
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    def rate(nbytes, sec):
        gbs = nbytes / sec / 1e9
        return {"GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBPS, 4)}

    back = torch.empty_like(nat)
    res = {"pack": {}, "unpack": {}, "axpy": {}, "dot": {}, "scale": {}, "nrm2": {},
           "pack_toward_zero": {}, "pack_to_odd": {}}
    for k in range(2, 9):
        x = flyte.pack((64, k), nat)
        res["pack"][k] = rate(n * (8 + k), timed(lambda: flyte.pack((64, k), nat, out=x)))
        res["unpack"][k] = rate(n * (k + 8), timed(lambda: flyte.unpack((64, k), x, out=back)))
        if k >= 3:
            y = x.clone()
            res["axpy"][k] = rate(3 * n * k, timed(lambda: flyte.axpy((64, k), 1.0 / 3.0, x, y)))
            r = torch.empty((), dtype=torch.float64, device=dev)
            res["dot"][k] = rate(2 * n * k, timed(lambda: flyte.dot((64, k), x, y, out=r)))
            res["scale"][k] = rate(2 * n * k, timed(lambda: flyte.scale((64, k), 1.0 + 2.0 ** -40, y)))
            res["nrm2"][k] = rate(n * k, timed(lambda: flyte.nrm2((64, k), x, out=r)))
            if k in (3, 5):
                res["pack_toward_zero"][k] = rate(n * (8 + k), timed(lambda: flyte.pack((64, k, 1), nat, out=x)))
                res["pack_to_odd"][k] = rate(n * (8 + k), timed(lambda: flyte.pack((64, k, 2), nat, out=x)))
            del y
        del x
    del nat, back
    nat32 = torch.empty(n, dtype=torch.float32, device=dev).uniform_(-1.0, 1.0, generator=g)
    back32 = torch.empty_like(nat32)
    for k in (2, 3):
        x = flyte.pack((32, k), nat32)
        res["pack"][f"b32k{k}"] = rate(n * (4 + k), timed(lambda: flyte.pack((32, k), nat32, out=x)))
        res["unpack"][f"b32k{k}"] = rate(n * (k + 4), timed(lambda: flyte.unpack((32, k), x, out=back32)))
        del x
    del nat32, back32
    torch.cuda.empty_cache()
    out.update(res)
    return out


def bench_batched(flyte, workloads, torch, dev, stream):
    """4096 independent GEMVs, m and n log-uniform in [64, 4096], formats uniform over
    all ten, entries U(-1,1): one persistent graph-launched kernel against the host
    loop of per-call launches and against that loop as a prebuilt graph."""
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
        y = torch.empty(d["m"], dtype=src.dtype, device=dev)
        items.append(flyte.GemvItem(f, d["m"], d["n"], d["lda"], A, x, y))
    del pool
    plan = flyte.BatchedGemv(items)
    t0 = time.perf_counter()
    plan.tune(reps=3)
    tune_s = time.perf_counter() - t0

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_persistent = timed(plan.launch, 5)
    ms_loop = timed(plan.loop, 3)
    ms_loop_graph = timed(plan.loop_graph, 3)
    nbytes = plan.nbytes
    out = {"count": len(items), "bytes": nbytes, "tune_s": round(tune_s, 2),
           "persistent_graph_ms": round(ms_persistent, 3),
           "persistent_graph_GBps": round(nbytes / (ms_persistent * 1e-3) / 1e9, 1),
           "loop_ms": round(ms_loop, 3), "loop_graph_ms": round(ms_loop_graph, 3),
           "speedup_vs_loop": round(ms_loop / ms_persistent, 3),
           "speedup_vs_loop_graph": round(ms_loop_graph / ms_persistent, 3)}
    plan.close()
    del items
    torch.cuda.empty_cache()
    return out


def bench_gemm(flyte, workloads, torch, np, dev, stream):
    """TFLOP/s of the GEMM paths (2*M*N*K useful flop per call), with the vendor
    library's bfloat16 and FP64 GEMMs at the same sizes beside them."""
    out = {}

    def timed(fn, reps, warm=1):
        # untimed calls first: the GPU clock takes a few milliseconds of load to settle
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps

    g = torch.Generator(device=dev)
    g.manual_seed(workloads.SEED_BASE + 2)
    Mg = 8192
    for k, name, flags in [(2, "bf16", 0), (3, "three_product", 0), (3, "four_product", flyte.GEMM_FOUR_PRODUCTS)]:
        Av = torch.empty(Mg * Mg, dtype=torch.float32, device=dev).normal_(generator=g)
        Bv = torch.empty(Mg * Mg, dtype=torch.float32, device=dev).normal_(generator=g)
        Ap, Bp = flyte.pack((32, k), Av), flyte.pack((32, k), Bv)
        del Av, Bv
        C = torch.empty(Mg * Mg, dtype=torch.float32, device=dev)
        ms = timed(lambda: flyte.gemm((32, k), (32, k), (32, 4), Mg, Mg, Mg, Ap, Bp, C, flags=flags), 10, warm=10)
        out[name] = {"M": Mg, "N": Mg, "K": Mg, "ms": round(ms, 3),
                     "TFLOPs": round(2.0 * Mg ** 3 / (ms * 1e-3) / 1e12, 1)}
        del Ap, Bp, C
    # the vendor library's bfloat16 GEMM at the same size (context, not a path of this library)
    a16 = torch.empty(Mg, Mg, dtype=torch.float32, device=dev).normal_(generator=g).bfloat16()
    b16 = torch.empty(Mg, Mg, dtype=torch.float32, device=dev).normal_(generator=g).bfloat16()
    ms = timed(lambda: torch.matmul(a16, b16), 10, warm=10)
    out["vendor_bf16_matmul"] = {"M": Mg, "N": Mg, "K": Mg, "ms": round(ms, 3),
                                 "TFLOPs": round(2.0 * Mg ** 3 / (ms * 1e-3) / 1e12, 1)}
    del a16, b16
    g.manual_seed(workloads.SEED_BASE + 4)
    Mf = 16384
    for k in (5, 6, 3):
        Av = torch.empty(Mf * Mf, dtype=torch.float64, device=dev).normal_(generator=g)
        Ap = flyte.pack((64, k), Av)
        Av.normal_(generator=g)
        Bp = flyte.pack((64, k), Av)
        del Av
        C = torch.empty(Mf * Mf * k, dtype=torch.uint8, device=dev)
        ms = timed(lambda: flyte.gemm((64, k), (64, k), (64, k), Mf, Mf, Mf, Ap, Bp, C), 2)
        out[f"fp64_k{k}"] = {"M": Mf, "N": Mf, "K": Mf, "ms": round(ms, 2),
                             "TFLOPs": round(2.0 * Mf ** 3 / (ms * 1e-3) / 1e12, 2)}
        del Ap, Bp, C
    # the vendor library's FP64 GEMM at the same size (native FP64 operands and C)
    a64 = torch.empty(Mf, Mf, dtype=torch.float64, device=dev).normal_(generator=g)
    b64 = torch.empty(Mf, Mf, dtype=torch.float64, device=dev).normal_(generator=g)
    ms = timed(lambda: torch.matmul(a64, b64), 2)
    out["vendor_fp64_matmul"] = {"M": Mf, "N": Mf, "K": Mf, "ms": round(ms, 2),
                                 "TFLOPs": round(2.0 * Mf ** 3 / (ms * 1e-3) / 1e12, 2)}
    del a64, b64
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    sys.exit(main())
