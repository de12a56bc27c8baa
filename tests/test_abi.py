"""Host-side checks of the C ABI (no GPU needed).

* libflyte.so loads and exports every function declared in include/flyte.h;
* argument errors are reported by status code, with a detail string, before
  anything is launched (invalid formats, null and misaligned pointers, bad
  leading dimensions, unsupported GEMM combinations, bad batch descriptors);
* the autotuner cache round-trips through its JSON file.
"""
from __future__ import annotations

import ctypes
import os
import re

import pytest

from paper_1601_07789_amd import flyte

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(fb_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    return flyte.load()


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(lib):
    assert flyte.status_name(0) == "FB_OK"
    assert flyte.status_name(4) == "FB_ERR_UNSUPPORTED"


def st(code):
    return code, flyte.last_error()


FAKE = 0x10000          # never dereferenced: validation fails first
MISALIGNED = 0x10002


def F(base, k, rnd=0, reserved=0):
    return flyte.fb_format(base, k, rnd, reserved)


def test_codec_argument_errors(lib):
    assert st(lib.fb_pack(F(32, 5), FAKE, FAKE, 10, None))[0] == flyte.FB_ERR_FORMAT
    assert st(lib.fb_pack(F(64, 1), FAKE, FAKE, 10, None))[0] == flyte.FB_ERR_FORMAT
    assert st(lib.fb_unpack(F(16, 2), FAKE, FAKE, 10, None))[0] == flyte.FB_ERR_FORMAT
    code, msg = st(lib.fb_pack(F(64, 5), None, FAKE, 10, None))
    assert code == flyte.FB_ERR_ARG and "null" in msg
    assert lib.fb_unpack(F(64, 5), MISALIGNED, FAKE, 10, None) == flyte.FB_ERR_ALIGN
    assert lib.fb_axpy(F(64, 3), 10, 1.0, FAKE, MISALIGNED, None) == flyte.FB_ERR_ALIGN
    assert lib.fb_dot(F(64, 3), 10, FAKE, FAKE, None, None) == flyte.FB_ERR_ARG
    assert lib.fb_dot(F(64, 3), 10, FAKE, FAKE, MISALIGNED, None) == flyte.FB_ERR_ALIGN
    assert lib.fb_pack(F(64, 5, 3), FAKE, FAKE, 10, None) == flyte.FB_ERR_FORMAT       # bad rounding mode
    assert lib.fb_pack(F(64, 5, 0, 1), FAKE, FAKE, 10, None) == flyte.FB_ERR_FORMAT    # reserved set
    assert lib.fb_scale(F(64, 5), 10, 2.0, MISALIGNED, None) == flyte.FB_ERR_ALIGN
    assert lib.fb_nrm2(F(64, 5), 10, FAKE, None, None) == flyte.FB_ERR_ARG
    assert lib.fb_scale(F(32, 2, 2), 0, 2.0, None, None) == flyte.FB_OK
    # n = 0 is valid and launches nothing (null data pointers allowed)
    assert lib.fb_pack(F(64, 5), None, None, 0, None) == flyte.FB_OK
    assert lib.fb_axpy(F(32, 3), 0, 2.0, None, None, None) == flyte.FB_OK


def test_gemv_argument_errors(lib):
    assert lib.fb_gemv(F(64, 9), 4, 4, FAKE, 4, FAKE, FAKE, None) == flyte.FB_ERR_FORMAT
    assert lib.fb_gemv(F(64, 5), -1, 4, FAKE, 4, FAKE, FAKE, None) == flyte.FB_ERR_ARG
    assert lib.fb_gemv(F(64, 5), 4, 8, FAKE, 4, FAKE, FAKE, None) == flyte.FB_ERR_ARG        # lda < n
    assert lib.fb_gemv(F(64, 5), 4, 3, FAKE, 3, FAKE, FAKE, None) == flyte.FB_ERR_ALIGN      # 15-byte rows
    assert lib.fb_gemv(F(64, 5), 4, 4, MISALIGNED, 4, FAKE, FAKE, None) == flyte.FB_ERR_ALIGN
    assert lib.fb_gemv(F(64, 5), 4, 4, None, 4, FAKE, FAKE, None) == flyte.FB_ERR_ARG
    assert lib.fb_gemv_config(F(64, 5), 4, 4, FAKE, 4, FAKE, FAKE, 99, None) == flyte.FB_ERR_ARG
    assert lib.fb_gemv(F(64, 5), 0, 4, None, 4, None, None, None) == flyte.FB_OK            # m = 0
    assert lib.fb_gemv_ex(F(64, 5), F(32, 3), 0, 4, 4, FAKE, 4, FAKE, FAKE, None) == flyte.FB_ERR_FORMAT
    assert lib.fb_gemv_ex(F(64, 5), F(64, 3), 2, 4, 4, FAKE, 4, FAKE, FAKE, None) == flyte.FB_ERR_ARG
    assert lib.fb_gemv_ex(F(64, 5), F(64, 3, 3), 0, 4, 4, FAKE, 4, FAKE, FAKE, None) == flyte.FB_ERR_FORMAT
    assert lib.fb_dot_packed(F(64, 5), F(32, 2), 4, FAKE, FAKE, FAKE, None) == flyte.FB_ERR_FORMAT
    # the transposed GEMV writes its n outputs even when m = 0, so y is checked then too
    assert lib.fb_gemv_ex(F(64, 8), F(64, 8), 1, 0, 4, None, 4, None, None, None) == flyte.FB_ERR_ARG
    assert lib.fb_gemv_ex(F(64, 8), F(64, 8), 1, 0, 4, None, 4, None, MISALIGNED, None) == flyte.FB_ERR_ALIGN


def test_gemm_argument_errors(lib):
    # every call below fails validation before anything is launched (the
    # pointers are never dereferenced)
    args = (128, 128, 64, FAKE, 64, FAKE, 128, FAKE, 128, None)
    assert lib.fb_gemm(F(32, 2), F(32, 3), F(32, 4), *args) == flyte.FB_ERR_UNSUPPORTED
    assert lib.fb_gemm(F(64, 7), F(32, 2), F(64, 7), *args) == flyte.FB_ERR_UNSUPPORTED
    assert lib.fb_gemm(F(64, 3), F(64, 3), F(32, 4), *args) == flyte.FB_ERR_UNSUPPORTED
    assert lib.fb_gemm(F(32, 2), F(32, 2), F(64, 8), *args) == flyte.FB_ERR_UNSUPPORTED
    assert lib.fb_gemm(F(64, 5), F(64, 6), F(64, 5), *args) == flyte.FB_ERR_UNSUPPORTED
    assert lib.fb_gemm(F(64, 5), F(64, 5), F(64, 5), 128, 128, 64, FAKE, 32, FAKE, 128, FAKE, 128,
                       None) == flyte.FB_ERR_ARG                                             # lda < K
    assert lib.fb_gemm(F(64, 5), F(64, 5), F(64, 5), 128, 128, 64, MISALIGNED, 64, FAKE, 128, FAKE, 128,
                       None) == flyte.FB_ERR_ALIGN
    assert lib.fb_gemm(F(64, 5), F(64, 5), F(64, 5), 128, 128, 3, FAKE, 3, FAKE, 128, FAKE, 128,
                       None) == flyte.FB_ERR_ALIGN                                           # 15-byte rows of A
    assert lib.fb_gemm(F(32, 3), F(32, 3), F(32, 4), 5, 7, 9, FAKE, 9, FAKE, 8, FAKE, 7,
                       None) == flyte.FB_ERR_ALIGN                                           # 27-byte rows of A
    assert lib.fb_gemm(F(64, 5), F(64, 5), F(64, 5), 0, 128, 64, None, 64, None, 128, None, 128,
                       None) == flyte.FB_OK
    assert lib.fb_gemm(F(64, 5), F(64, 5), F(64, 5), 128, 128, 64, None, 64, FAKE, 128, FAKE, 128,
                       None) == flyte.FB_ERR_ARG                                             # null A
    assert lib.fb_gemm(F(32, 2), F(32, 2), F(32, 4), -1, 128, 64, FAKE, 64, FAKE, 128, FAKE, 128,
                       None) == flyte.FB_ERR_ARG                                             # negative M
    # flags: all products only for split operands; FP64 only for binary64; unknown bits
    assert lib.fb_gemm_ex(F(32, 2), F(32, 2), F(32, 4), *args[:-1], 1, None) == flyte.FB_ERR_UNSUPPORTED
    assert lib.fb_gemm_ex(F(64, 5), F(64, 5), F(64, 5), *args[:-1], 1, None) == flyte.FB_ERR_UNSUPPORTED
    assert lib.fb_gemm_ex(F(64, 3), F(64, 3), F(64, 3), *args[:-1], 3, None) == flyte.FB_ERR_UNSUPPORTED
    assert lib.fb_gemm_ex(F(32, 3), F(32, 3), F(32, 4), *args[:-1], 2, None) == flyte.FB_ERR_UNSUPPORTED
    assert lib.fb_gemm_ex(F(32, 3), F(32, 3), F(32, 4), *args[:-1], 4, None) == flyte.FB_ERR_ARG


def test_batched_plan_rejects_bad_descriptor(lib):
    D = flyte.fb_gemv_desc
    arr = (D * 2)()
    arr[0] = D(flyte.fmt((64, 5)), 4, 4, 0, 4, FAKE, FAKE, FAKE)
    arr[1] = D(flyte.fmt((64, 5)), 4, 4, 0, 3, FAKE, FAKE, FAKE)   # lda < n
    plan = ctypes.c_void_p()
    code = lib.fb_gemv_batched_plan(arr, 2, ctypes.byref(plan))
    assert code == flyte.FB_ERR_ARG and "descriptor 1" in flyte.last_error()
    assert not plan.value
    assert lib.fb_gemv_batched_plan(arr, -1, ctypes.byref(plan)) == flyte.FB_ERR_ARG
    assert lib.fb_gemv_batched_launch(None, None) == flyte.FB_ERR_ARG
    lib.fb_plan_destroy(None)


def test_tune_cache_round_trip(tmp_path):
    flyte.tune_clear()
    assert flyte.tune_lookup((64, 5), 8192, 8192) == -1
    flyte.tune_record((64, 5), 8192, 8192, 3, 57.5)
    flyte.tune_record((32, 2), 100, 3000, 9, 4.0)
    assert flyte.tune_lookup((64, 5), 8200, 9000) == 3          # same floor(log2) buckets
    path = str(tmp_path / "tiles.json")
    flyte.tune_save(path)
    flyte.tune_clear()
    assert flyte.tune_lookup((64, 5), 8192, 8192) == -1
    flyte.tune_load(path)
    assert flyte.tune_lookup((64, 5), 8192, 8192) == 3
    assert flyte.tune_lookup((32, 2), 100, 3000) == 9
    with pytest.raises(flyte.FlyteError):
        flyte.tune_record((64, 5), 10, 10, 999, 1.0)
    bad = tmp_path / "bad.json"
    bad.write_text('{"entries": [{"base": 64, "k": 12}]}')
    with pytest.raises(flyte.FlyteError):
        flyte.tune_load(str(bad))
    flyte.tune_clear()


def test_gemv_config_table():
    n = flyte.gemv_num_configs()
    assert n >= 10
    infos = [flyte.gemv_config_info(c) for c in range(n)]
    assert all(i["lanes_per_row"] in (8, 16, 32, 64) for i in infos)
    assert flyte.load().fb_gemv_config_info(n, None, None, None) == 0


def test_tune_cache_concurrent_threads():
    """Threads recording and looking up tile choices at once (the foreign calls run without
    the interpreter lock): every lookup returns a value some thread recorded for that
    bucket, and the cache ends with one entry per bucket."""
    import threading
    flyte.tune_clear()
    errors = []

    def worker(t):
        try:
            for i in range(2000):
                m = 1 << (4 + (i % 8))
                flyte.tune_record((64, 3 + (t % 6)), m, 4096, (t + i) % flyte.gemv_num_configs(), 1.0)
                got = flyte.tune_lookup((64, 3 + (t % 6)), m, 4096)
                if not (0 <= got < flyte.gemv_num_configs()):
                    errors.append((t, i, got))
        except Exception as exc:     # noqa: BLE001 -- collected and reported below
            errors.append(exc)

    threads = [threading.Thread(target=worker, args=(t,)) for t in range(8)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors, errors[:3]
    for kk in range(3, 9):
        for e in range(8):
            assert 0 <= flyte.tune_lookup((64, kk), 1 << (4 + e), 4096) < flyte.gemv_num_configs()
    flyte.tune_clear()
