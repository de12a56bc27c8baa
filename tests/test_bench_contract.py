"""Host-side checks of bench.py (no GPU needed).

* `--gpus N` with N > 1 exits with status 2 and says that only one GPU is
  measured, before touching the device.
* The committed HBM-counter summary of the GEMV matches the current GEMV sources
  and the committed tile cache, so the benchmark reports measured traffic rather
  than null (a changed GEMV kernel or tile choice needs new counter passes).
* The provenance entry names this repository's commit and a source hash.
"""
from __future__ import annotations

import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counter_summary_matches_sources_and_tiles():
    from paper_1601_07789_amd import flyte
    bench = load_bench()
    flyte.tune_clear()
    try:
        flyte.tune_load(bench.DEFAULT_TILES)
        tiles = {k: flyte.tune_lookup((64, k), bench.M, bench.N) for k in bench.KS}
    finally:
        flyte.tune_clear()
    assert all(t >= 0 for t in tiles.values()), tiles
    traffic = bench.measured_traffic(tiles)
    assert traffic is not None, "profiles/gemv_8192x8192_k3-8_hbm_counters.md is stale"
    algorithmic = sum(bench.gemv_bytes(k) for k in bench.KS)
    assert 0.99 * algorithmic <= traffic <= 1.05 * algorithmic


def test_provenance_names_this_tree():
    bench = load_bench()
    p = bench.provenance()
    assert len(p["sources_sha256"]) == 16
    r = subprocess.run(["git", "rev-parse", "--show-toplevel", "HEAD"], cwd=ROOT, capture_output=True, text=True)
    out = r.stdout.split()
    if r.returncode == 0 and len(out) == 2 and os.path.realpath(out[0]) == os.path.realpath(ROOT):
        assert p["git_commit"] == out[1]
    else:
        assert p["git_commit"] is None
