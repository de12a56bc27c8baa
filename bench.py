#!/usr/bin/env python3
"""Benchmark of the k-byte GEMV hot path on one MI355X.

Workload: y = A x with A 8192 x 8192 row-major, stored in the binary64-derived
k-byte formats k = 3..8 (entries U(-1,1) packed on the device by fb_pack), x
and y FP64, FP64 accumulation.  One step runs, for every k, one GEMV over each
of R rotating copies of A (R * size(A) >= 1 GiB, so the 256 MB last-level
cache holds none of the A being read).  k = 8 is the FP64-stored baseline; the
vendor FP64 GEMV (torch.mv -> rocBLAS) is timed beside it.

value = algorithmic bytes of every GEMV in the timed region / wall time.
In every step HIP events on the launch stream bracket each k's R back-to-back
launches (at least 100 launches per k with the default 25 steps); per k the
median over steps of the mean launch time and the overall mean are reported,
and the roofline entry divides the algorithmic bytes by the mean, against the
8 TB/s HBM peak, with the HBM
traffic measured by the committed counter profile when it matches the kernels
and tiles in use.  After the timed region (reported under "detail"): the
transposed GEMV, the codec and BLAS-1 kernels at 2^28 elements and the
round-trip workload at 2^20, the batched workload (4096 mixed GEMVs), and the
GEMMs (BF16, 3- and 4-product, FP64 with a k-byte C) with their errors against
FP64 references and the vendor library's GEMMs beside them.  cpu_baseline times
the oracle's GEMV on all host cores and on one thread; detail.cpu_oracle times
the oracle on the other workloads (bounded samples, extrapolations labelled).
detail.provenance names the input seeds, the git commit (when the tree is a
repository) and a hash of the kernel sources.

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
    ap.add_argument("--steps", type=int, default=25)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rotate", type=int, default=0, help="A copies per k (0: enough for >= 1 GiB)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gemm", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-blas1", action="store_true")
    ap.add_argument("--retune", action="store_true",
                    help="rank the GEMV tiles with rotating buffers over interleaved rounds instead of "
                         "loading the committed cache")
    ap.add_argument("--tune-rounds", type=int, default=7, help="interleaved rounds of --retune")
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

    # ------------------------------------------------------------ tile choice
    tiles = {}
    tuning = None
    if not args.retune and os.path.exists(args.tune_cache):
        flyte.tune_load(args.tune_cache)
        log(f"tiles loaded from {args.tune_cache}")
    if args.retune:
        log(f"ranking GEMV tiles with rotating buffers over {args.tune_rounds} interleaved rounds")
        tuning = retune(flyte, torch, np, stream, A, R, x, y, args.tune_rounds)
        for k in KS:
            best = tuning[k]["best"]
            flyte.tune_record((64, k), M, N, best, tuning[k]["us"][best])
            tiles[k] = best
        flyte.tune_save(args.tune_cache)
        log(f"tiles saved to {args.tune_cache}")
    for k in KS:
        tiles.setdefault(k, flyte.tune_lookup((64, k), M, N))

    # ------------------------------------------------------------ timed GEMV sweep
    # Events bracket each k's R back-to-back launches of a step (an event between
    # every launch would add its own gap to each launch).
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
    step_events = [{k: (ev(), ev()) for k in KS} for _ in range(args.steps)]
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(step_events[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # per step and k: the mean time of that step's R launches
    launch_ms = {k: [step_events[s][k][0].elapsed_time(step_events[s][k][1]) / R[k] for s in range(args.steps)]
                 for k in KS}
    bytes_per_step = sum(R[k] * gemv_bytes(k) for k in KS)
    ms_per_step = 1000.0 * wall / args.steps
    value = bytes_per_step / (wall / args.steps) / 1e9

    per_k = {}
    for k in KS:
        mean_us = 1000.0 * float(np.mean(launch_ms[k]))
        med_us = 1000.0 * float(np.median(launch_ms[k]))
        gbs = gemv_bytes(k) / (med_us * 1e-6) / 1e9
        per_k[k] = {"us": round(med_us, 2), "us_mean": round(mean_us, 2), "launches": args.steps * R[k],
                    "GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBPS, 4), "tile": tiles[k]}

    # ------------------------------------------------------------ vendor FP64 GEMV (rocBLAS via torch.mv)
    log("timing vendor FP64 GEMV")
    it = [0]

    def vendor():
        torch.mv(A64[it[0] % len(A64)], x, out=y)
        it[0] += 1

    vendor_us = 1000.0 * median_ms(torch, stream, vendor, 100, warm=len(A64), group=len(A64))
    fp64_stored_us = min(vendor_us, per_k[8]["us"])
    for k in KS:
        per_k[k]["speedup_vs_fp64_stored"] = round(fp64_stored_us / per_k[k]["us"], 3)
        per_k[k]["ideal_8_over_k"] = round(8.0 / k, 3)

    # the transposed GEMV (y = A^T x) on the same matrices
    trans = {}
    yt = torch.empty(N, dtype=torch.float64, device=dev)
    for k in KS:
        it[0] = 0

        def tgemv():
            flyte.gemv_ex((64, k), (64, 8), True, A[k][it[0] % R[k]], M, N, x, y=yt)
            it[0] += 1

        us = 1000.0 * median_ms(torch, stream, tgemv, 25 * R[k], warm=R[k], group=R[k])
        trans[k] = {"us": round(us, 2), "GBps": round(gemv_bytes(k) / (us * 1e-6) / 1e9, 1)}

    # roofline over the GEMV launches (one kernel template, six formats): mean launch times
    tot_bytes = sum(gemv_bytes(k) for k in KS)
    tot_us = sum(per_k[k]["us_mean"] for k in KS)
    achieved = tot_bytes / (tot_us * 1e-6) / 1e9
    traffic = measured_traffic(tiles)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": "flyte::k_gemv (binary64-derived k=3..8, one launch per k; "
                          "achieved = sum of algorithmic bytes / sum of mean launch durations)"}
    del A64

    # ------------------------------------------------------------ measured stream references
    stream_ref = measure_streams(torch, dev, stream)

    # ------------------------------------------------------------ CPU baseline: the oracle's GEMV
    cpu = None
    if not args.no_cpu_baseline:
        log("oracle GEMV on the host (all cores, then one thread)")
        cpu = cpu_baseline(A, x, np)

    detail = {"per_k": per_k, "transposed_per_k": trans, "vendor_fp64_gemv_us": round(vendor_us, 2), "rotate": R,
              "bytes_per_step": bytes_per_step, "stream_reference": stream_ref,
              "gemv_frac_of_measured_read_stream": round(achieved / stream_ref["read_GBps"], 4)}
    if tuning is not None:
        detail["tuning"] = {k: {"best": v["best"], "rounds": v["rounds"],
                                "top3_us": sorted(v["us"].values())[:3]} for k, v in tuning.items()}
    del A
    torch.cuda.empty_cache()
    oracle_times = {}
    if not args.no_gemm:
        try:
            detail["gemm"] = bench_gemm(flyte, workloads, torch, np, dev, stream,
                                        None if args.no_cpu_baseline else oracle_times)
        except Exception as e:   # reported, not hidden: the GEMV line stands on its own
            detail["gemm"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_blas1:
        try:
            detail["blas1"] = bench_blas1(flyte, workloads, torch, dev, stream)
            detail["round_trip_2e20"] = bench_round_trip(flyte, workloads, torch, np, dev, stream,
                                                         None if args.no_cpu_baseline else oracle_times)
        except Exception as e:
            detail["blas1"] = {"error": f"{type(e).__name__}: {e}"}
    if not args.no_batched:
        try:
            detail["batched"] = bench_batched(flyte, workloads, torch, np, dev, stream,
                                              None if args.no_cpu_baseline else oracle_times)
        except Exception as e:
            detail["batched"] = {"error": f"{type(e).__name__}: {e}"}
    if oracle_times:
        detail["cpu_oracle"] = oracle_times

    prov["seeds"] = {"gemv_A": workloads.SEED_BASE + 1, "gemv_x": workloads.SEED_BASE + 101,
                     "gemm_b32": workloads.SEED_BASE + 2, "batched": workloads.SEED_BASE + 3,
                     "gemm_f64": workloads.SEED_BASE + 4, "blas1": workloads.SEED_BASE + 1,
                     "round_trip": workloads.SEED_BASE}
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


def ev():
    import torch
    return torch.cuda.Event(enable_timing=True)


def median_ms(torch, stream, fn, calls, warm=3, group=1):
    """Per-call time (ms): `calls` calls after `warm` untimed ones (the GPU may have
    idled before), in groups of `group` back-to-back calls bracketed by HIP events on
    `stream`; the median over the groups of the mean call time in each group (an
    event pair around every short call would add its own gap to each)."""
    import numpy as np
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    evs = [(ev(), ev()) for _ in range(max(1, calls // group))]
    for e0, e1 in evs:
        e0.record(stream)
        for _ in range(group):
            fn()
        e1.record(stream)
    torch.cuda.synchronize()
    return float(np.median([e0.elapsed_time(e1) / group for e0, e1 in evs]))


def retune(flyte, torch, np, stream, A, R, x, y, rounds):
    """Ranks every GEMV tile per k: in each round every candidate (in a seeded
    shuffled order) runs 2 R launches over the rotating copies, timed with events;
    a candidate's time is its median over the rounds, and the fastest wins.
    Interleaving the rounds keeps the drift of clocks and of the memory system
    between candidates out of the ranking (single passes differ by a few percent)."""
    out = {}
    ncfg = flyte.gemv_num_configs()
    rng = np.random.default_rng(1601)
    for k in KS:
        times = {c: [] for c in range(ncfg)}
        for rnd in range(rounds):
            for c in rng.permutation(ncfg):
                c = int(c)
                for r in range(R[k]):
                    flyte.gemv((64, k), A[k][r], M, N, x, y=y, config=c)
                e0, e1 = ev(), ev()
                e0.record(stream)
                for rep in range(2):
                    for r in range(R[k]):
                        flyte.gemv((64, k), A[k][r], M, N, x, y=y, config=c)
                e1.record(stream)
                e1.synchronize()
                times[c].append(1000.0 * e0.elapsed_time(e1) / (2 * R[k]))
        us = {c: round(float(np.median(v)), 2) for c, v in times.items()}
        best = min(us, key=us.get)
        out[k] = {"best": best, "us": us, "rounds": rounds}
        log(f"  k={k}: tile {best} at {us[best]} us")
    return out


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


def cpu_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def parallel_rows(fn, m, threads):
    """Runs fn(r0, r1) over `threads` contiguous row blocks of [0, m) on a thread pool
    (the oracle's foreign calls release the interpreter lock) and returns the wall time."""
    from concurrent.futures import ThreadPoolExecutor
    bounds = [(m * t // threads, m * (t + 1) // threads) for t in range(threads)]
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(lambda b: fn(*b), bounds))
    return time.perf_counter() - t0


def cpu_baseline(A, x, np):
    """The oracle's naive GEMV (sequential fma per row) on the host, unchanged, over
    the full 8192 x 8192 matrix of each k: with its rows split into one block per
    host thread (all cores, the reported value), and on one thread; each repeated to
    about 1 s (all cores) and 1.5 s (one thread) per k."""
    import oracle
    orc = oracle.default()
    xh = x.cpu().numpy()
    nth = cpu_threads()
    res = {}
    for label, threads, budget in (("all", nth, 1.0), ("one", 1, 1.5)):
        total_bytes, total_s, passes = 0, 0.0, {}
        for k in KS:
            Ah = A[k][0].cpu().numpy()

            def rows(r0, r1, Ah=Ah, k=k):
                orc.gemv_naive(64, k, r1 - r0, N, Ah[r0 * N * k:r1 * N * k], N, xh)

            p, spent = 0, 0.0
            while spent < budget:
                spent += parallel_rows(rows, M, threads)
                p += 1
            total_bytes += p * gemv_bytes(k)
            total_s += spent
            passes[k] = p
        res[label] = {"GBps": round(total_bytes / total_s / 1e9, 4), "threads": threads, "passes": passes,
                      "seconds": round(total_s, 1)}
    return {"value": res["all"]["GBps"], "unit": "GB/s", "cores": nth, "kind": "oracle",
            "sample": f"oracle fbo_gemv_naive, full 8192x8192 GEMV per k = 3..8, rows split into {nth} blocks "
                      f"on {nth} threads, passes per k = {res['all']['passes']} ({res['all']['seconds']} s wall); "
                      f"one thread: {res['one']['GBps']} GB/s (passes {res['one']['passes']}, "
                      f"{res['one']['seconds']} s)",
            "single_thread": {"value": res["one"]["GBps"], "unit": "GB/s", "cores": 1},
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




def rate(nbytes, sec):
    gbs = nbytes / sec / 1e9
    return {"GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBPS, 4)}


def bench_blas1(flyte, workloads, torch, dev, stream):
    """Streaming codec and BLAS-1 kernels on n = 2^28 elements (the 2 GiB FP64 side
    and every packed array exceed the 256 MB last-level cache): algorithmic GB/s
    (100 calls in groups of 4, median of the group means) and fraction of 8 TB/s.  pack: n(W+k) bytes, unpack:
    n(k+W), axpy: 3nk, dot: 2nk, scale (in place): 2nk, nrm2: nk."""
    n = 1 << 28
    calls = 100
    g = torch.Generator(device=dev)
    g.manual_seed(workloads.SEED_BASE + 1)
    nat = torch.empty(n, dtype=torch.float64, device=dev).uniform_(-1.0, 1.0, generator=g)
    out = {"n": n, "calls": calls}

    def timed(fn):
        return median_ms(torch, stream, fn, calls, group=4) * 1e-3

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
    # the in-tree read+write ceiling: pack to {64,8} cuts no bits (the identity
    # codec), so it is a plain read+write dword stream with the same chunked grid
    # and 16-byte lane units as the codec and BLAS-1 kernels
    ceil = res["pack"][8]["GBps"]
    out["stream_ceiling"] = {"kernel": "k_pack {64,8} (identity: a plain 16-byte-unit read+write stream, same grid)",
                             "GBps": ceil, "frac_hbm": round(ceil / HBM_PEAK_GBPS, 4)}
    for op in ("pack", "unpack", "axpy", "scale"):
        for key, v in res[op].items():
            v["frac_of_stream_ceiling"] = round(v["GBps"] / ceil, 4)
    out.update(res)
    return out


def bench_round_trip(flyte, workloads, torch, np, dev, stream, oracle_times):
    """The round-trip workload: 2^20 binary64 values from the mixed population (90%
    N(0,1) 2^U(-60,60), 10% specials), for every k = 2..8: pack, unpack of the
    packed result and the dot of two packed vectors, on the GPU (median of 100
    calls; 8-16 MB stay in the last-level cache, so these are latency-bound
    times, not bandwidth claims) and, with the oracle timed beside it, on the host
    (one thread, whole arrays)."""
    import oracle
    n = 1 << 20
    xb = workloads.mixed_binary64(n, workloads.SEED_BASE)
    yb = workloads.mixed_binary64(n, workloads.SEED_BASE + 100)
    xd = torch.from_numpy(xb.view(np.float64)).to(dev)
    yd = torch.from_numpy(yb.view(np.float64)).to(dev)
    back = torch.empty_like(xd)
    r = torch.empty((), dtype=torch.float64, device=dev)
    gpu = {}
    cpu = {}
    orc = oracle.default() if oracle_times is not None else None
    for k in range(2, 9):
        px = flyte.pack((64, k), xd)
        py = flyte.pack((64, k), yd)
        t_pack = median_ms(torch, stream, lambda: flyte.pack((64, k), xd, out=px), 200, group=10)
        t_unpack = median_ms(torch, stream, lambda: flyte.unpack((64, k), px, out=back), 200, group=10)
        t_dot = median_ms(torch, stream, lambda: flyte.dot((64, k), px, py, out=r), 200, group=10)
        gpu[k] = {"pack_us": round(1000 * t_pack, 2), "unpack_us": round(1000 * t_unpack, 2),
                  "dot_us": round(1000 * t_dot, 2)}
        if orc is not None:
            qy = orc.pack(64, k, yb.view(np.float64))
            t0 = time.perf_counter()
            q = orc.pack(64, k, xb.view(np.float64))
            t1 = time.perf_counter()
            orc.unpack(64, k, q)
            t2 = time.perf_counter()
            orc.dot_naive(64, k, q, qy)
            t3 = time.perf_counter()
            cpu[k] = {"pack_us": round(1e6 * (t1 - t0), 1), "unpack_us": round(1e6 * (t2 - t1), 1),
                      "dot_us": round(1e6 * (t3 - t2), 1)}
        del px, py
    del xd, yd, back
    if orc is not None:
        oracle_times["round_trip_2e20"] = {"threads": 1, "per_k": cpu,
                                           "sample": "the whole workload: 2^20 values per k, each op once"}
    return {"n": n, "per_k": gpu}


def bench_batched(flyte, workloads, torch, np, dev, stream, oracle_times):
    """4096 independent GEMVs, m and n log-uniform in [64, 4096], formats uniform over
    all ten, entries U(-1,1): one persistent graph-launched kernel (median of 100
    launches) against the host loop of per-call launches and against that loop as a
    prebuilt graph (median of 20 each).  With the oracle: its naive GEMV over the
    first 512 descriptors on all host threads, extrapolated to the batch by bytes."""
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

    ms_persistent = median_ms(torch, stream, plan.launch, 100)
    ms_loop = median_ms(torch, stream, plan.loop, 20, warm=1)
    ms_loop_graph = median_ms(torch, stream, plan.loop_graph, 20, warm=1)
    nbytes = plan.nbytes
    out = {"count": len(items), "bytes": nbytes, "tune_s": round(tune_s, 2),
           "persistent_graph_ms": round(ms_persistent, 3),
           "persistent_graph_GBps": round(nbytes / (ms_persistent * 1e-3) / 1e9, 1),
           "persistent_graph_frac_hbm": round(nbytes / (ms_persistent * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
           "loop_ms": round(ms_loop, 3), "loop_graph_ms": round(ms_loop_graph, 3),
           "speedup_vs_loop": round(ms_loop / ms_persistent, 3),
           "speedup_vs_loop_graph": round(ms_loop_graph / ms_persistent, 3)}
    plan.close()
    if oracle_times is not None:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        orc = oracle.default()
        sample = items[:512]
        host = [(it.f, it.m, it.n, it.lda, it.A.cpu().numpy(), it.x.cpu().numpy()) for it in sample]
        sbytes = sum(it.m * it.n * it.f[1] + (it.m + it.n) * it.f[0] // 8 for it in sample)
        nth = cpu_threads()
        t0 = time.perf_counter()
        with ThreadPoolExecutor(nth) as ex:
            list(ex.map(lambda h: orc.gemv_naive(h[0][0], h[0][1], h[1], h[2], h[4], h[3], h[5]), host))
        spent = time.perf_counter() - t0
        oracle_times["batched"] = {
            "threads": nth, "sample": "naive GEMV of the first 512 of the 4096 descriptors (one descriptor per "
                                      "task on a pool of host threads)",
            "sample_bytes": sbytes, "seconds": round(spent, 2), "GBps": round(sbytes / spent / 1e9, 3),
            "extrapolated_batch_ms": round(1e3 * spent * nbytes / sbytes, 1)}
    del items
    torch.cuda.empty_cache()
    return out


def gemm_errors(orc, np, fa, fc, M, N, K, Ah, Bh, C_rows, rows, exact_entries=128):
    """Errors of sampled rows of a GEMM result against references built from the
    oracle-unpacked operands:
      e1 = max |dC| / (|A||B|), e2 = ||dC||_F / ||C||_F, e3 = max |dC| / max |C|
    over the given full rows, the reference being the FP64 product of the unpacked
    operands (its own error, gamma_K(2^-53) |A||B|, is below 2e-12 |A||B| here), and
    e1 again on a few entries of those rows against the oracle's exact dot."""
    base, k = fa
    Bn = orc.unpack(base, k, Bh).astype(np.float64).reshape(K, N)
    An = np.stack([orc.unpack(base, k, Ah[r * K * k:(r + 1) * K * k]).astype(np.float64) for r in rows])
    ref = An @ Bn
    absref = np.abs(An) @ np.abs(Bn)
    d = np.abs(C_rows - ref)
    out = {"rows": [int(r) for r in rows], "e1": float(np.max(d / absref)),
           "e2": float(np.linalg.norm(d) / np.linalg.norm(ref)), "e3": float(np.max(d) / np.max(np.abs(ref)))}
    rng = np.random.default_rng(7)
    ii = np.asarray(rows)[rng.integers(0, len(rows), exact_entries)]
    jj = rng.integers(0, N, exact_entries)
    ce, cab = orc.gemm_entries(fa, fa, K, Ah, K, Bh, N, ii, jj)
    pos = {int(r): t for t, r in enumerate(rows)}
    got = np.array([C_rows[pos[int(i)], int(j)] for i, j in zip(ii, jj)])
    out["e1_exact_entries"] = float(np.max(np.abs(got - ce) / cab))
    out["method"] = (f"{len(rows)} full rows (first, last, seeded random) against the FP64 product of the "
                     f"oracle-unpacked operands; e1_exact_entries: {exact_entries} entries of those rows against "
                     f"the oracle's exact dot")
    return out, Bn


def bench_gemm(flyte, workloads, torch, np, dev, stream, oracle_times):
    """TFLOP/s of the GEMM paths (2*M*N*K useful flop per call; median of 10 calls at
    8192^3, 3 at 16384^3; binary64 k = 2..4 both on bfloat16 pieces and on FP64
    matrix cores), their errors e1, e2, e3 on sampled rows, the vendor
    library's bfloat16 and FP64 GEMMs at the same sizes beside them, and with the
    oracle: its naive GEMM timed on a block of rows on all host threads, the full
    time extrapolated from it."""
    import oracle
    orc = oracle.default()
    out = {}
    nth = cpu_threads()

    def tf(M, ms):
        return round(2.0 * M ** 3 / (ms * 1e-3) / 1e12, 2)

    def oracle_block(fa, Mfull, K, N, Ah, Bh, rows_block):
        def rows(r0, r1):
            orc.gemm_naive(fa, fa, r1 - r0, N, K, Ah[r0 * K * fa[1]:r1 * K * fa[1]], K, Bh, N)
        spent = parallel_rows(rows, rows_block, nth)
        flops = 2.0 * rows_block * N * K
        return {"threads": nth, "rows": rows_block, "seconds": round(spent, 2),
                "GFLOPs": round(flops / spent / 1e9, 3),
                "extrapolated_full_s": round(spent * Mfull / rows_block, 1),
                "sample": f"naive GEMM (sequential fma per entry) of rows 0..{rows_block - 1} of the "
                          f"{Mfull}^3 product; full time extrapolated by rows"}

    g = torch.Generator(device=dev)
    g.manual_seed(workloads.SEED_BASE + 2)
    Mg = 8192
    rng = np.random.default_rng(3)
    rows_g = [0, Mg - 1] + [int(r) for r in rng.integers(1, Mg - 1, 2)]
    for k, name, flags in [(2, "bf16", 0), (3, "three_product", 0), (3, "four_product", flyte.GEMM_FOUR_PRODUCTS)]:
        if name != "four_product":
            Av = torch.empty(Mg * Mg, dtype=torch.float32, device=dev).normal_(generator=g)
            Bv = torch.empty(Mg * Mg, dtype=torch.float32, device=dev).normal_(generator=g)
            Ap, Bp = flyte.pack((32, k), Av), flyte.pack((32, k), Bv)
            del Av, Bv
            Ah, Bh = Ap.cpu().numpy(), Bp.cpu().numpy()
        C = torch.empty(Mg * Mg, dtype=torch.float32, device=dev)
        ms = median_ms(torch, stream,
                       lambda: flyte.gemm((32, k), (32, k), (32, 4), Mg, Mg, Mg, Ap, Bp, C, flags=flags), 10, warm=10)
        entry = {"M": Mg, "N": Mg, "K": Mg, "ms": round(ms, 3), "TFLOPs": tf(Mg, ms)}
        C_rows = C.view(Mg, Mg)[torch.tensor(rows_g, device=dev)].cpu().numpy().astype(np.float64)
        entry["errors"], _ = gemm_errors(orc, np, (32, k), (32, 4), Mg, Mg, Mg, Ah, Bh, C_rows, rows_g)
        out[name] = entry
        if oracle_times is not None and name != "four_product":
            oracle_times[f"gemm_b32_k{k}"] = oracle_block((32, k), Mg, Mg, Mg, Ah, Bh, 2 * nth)
        del C
        if name != "three_product":
            del Ap, Bp
    # the vendor library's bfloat16 GEMM at the same size (context, not a path of this library)
    a16 = torch.empty(Mg, Mg, dtype=torch.float32, device=dev).normal_(generator=g).bfloat16()
    b16 = torch.empty(Mg, Mg, dtype=torch.float32, device=dev).normal_(generator=g).bfloat16()
    ms = median_ms(torch, stream, lambda: torch.matmul(a16, b16), 10, warm=10)
    out["vendor_bf16_matmul"] = {"M": Mg, "N": Mg, "K": Mg, "ms": round(ms, 3), "TFLOPs": tf(Mg, ms)}
    del a16, b16
    g.manual_seed(workloads.SEED_BASE + 4)
    Mf = 16384
    rows_f = [0, Mf - 1] + [int(r) for r in rng.integers(1, Mf - 1, 2)]
    # binary64 k = 5, 6 on FP64 matrix cores; k = 2, 3, 4 on bfloat16 pieces (the
    # default) and, beside them, on FP64 matrix cores (FB_GEMM_FP64)
    runs = [(5, "fp64_k5", 0), (6, "fp64_k6", 0), (3, "fp64_k3", flyte.GEMM_FP64), (3, "pieces_k3", 0),
            (2, "fp64_k2", flyte.GEMM_FP64), (2, "pieces_k2", 0), (4, "fp64_k4", flyte.GEMM_FP64), (4, "pieces_k4", 0)]
    cur = None
    for k, name, flags in runs:
        if cur != k:
            Ap = Bp = Ah = Bh = None
            torch.cuda.empty_cache()
            Av = torch.empty(Mf * Mf, dtype=torch.float64, device=dev).normal_(generator=g)
            Ap = flyte.pack((64, k), Av)
            Av.normal_(generator=g)
            Bp = flyte.pack((64, k), Av)
            del Av
            C = torch.empty(Mf * Mf * k, dtype=torch.uint8, device=dev)
            Ah, Bh = Ap.cpu().numpy(), Bp.cpu().numpy()
            cur = k
        ms = median_ms(torch, stream, lambda: flyte.gemm((64, k), (64, k), (64, k), Mf, Mf, Mf, Ap, Bp, C, flags=flags),
                       3, warm=1)
        entry = {"M": Mf, "N": Mf, "K": Mf, "ms": round(ms, 2), "TFLOPs": tf(Mf, ms),
                 "path": "bfloat16 pieces" if name.startswith("pieces") else "FP64 matrix cores"}
        Cb = C.view(Mf, Mf * k)[torch.tensor(rows_f, device=dev)].cpu().numpy()
        C_rows = np.stack([orc.unpack(64, k, Cb[t]) for t in range(len(rows_f))])
        entry["errors"], _ = gemm_errors(orc, np, (64, k), (64, k), Mf, Mf, Mf, Ah, Bh, C_rows, rows_f)
        entry["errors"]["c_format_half_ulp"] = 2.0 ** -(8 * k - 12 + 1)
        out[name] = entry
        if oracle_times is not None and name in ("fp64_k5", "fp64_k6"):
            oracle_times[f"gemm_b64_k{k}"] = oracle_block((64, k), Mf, Mf, Mf, Ah, Bh, nth)
    del Ap, Bp, C, Ah, Bh
    torch.cuda.empty_cache()
    # the vendor library's FP64 GEMM at the same size (native FP64 operands and C)
    a64 = torch.empty(Mf, Mf, dtype=torch.float64, device=dev).normal_(generator=g)
    b64 = torch.empty(Mf, Mf, dtype=torch.float64, device=dev).normal_(generator=g)
    ms = median_ms(torch, stream, lambda: torch.matmul(a64, b64), 3, warm=1)
    out["vendor_fp64_matmul"] = {"M": Mf, "N": Mf, "K": Mf, "ms": round(ms, 2), "TFLOPs": tf(Mf, ms)}
    del a64, b64
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    sys.exit(main())
