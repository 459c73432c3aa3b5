"""Host logic of the serving form (CPU only): the native pool allocator
(compiled alone with g++ from its header) and the admission target."""

import math
import os
import shutil
import subprocess
import tempfile

import pytest

serve = pytest.importorskip("paper_2207_06374_amd.serve")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_pool_allocator_first_fit_merge_peak_and_random_sequences():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "pool_alloc_check")
        # host code only: built with g++ under the address and undefined-behaviour sanitizers
        subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Werror", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "paper_2207_06374_amd", "csrc"),
                        os.path.join(ROOT, "tests", "pool_alloc_check.cpp"), "-o", exe], check=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
        assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout


def test_welch_target():
    assert serve.welch_bound(16, 8) == math.sqrt(8 / (8 * 15))
    assert serve.welch_bound(4, 8) == 0.0
    assert math.isnan(serve.welch_bound(1, 8))


def test_footprint_and_server_argument_checks_without_device():
    """The footprint is workspace + frame + scalars, each rounded to 256
    bytes; the server rejects bad parameters before touching a device."""
    import ctypes

    from paper_2207_06374_amd import _abi, default_params, workspace_bytes
    p = default_params(300, 16, candidates=32, mode="bf16", recheck_topk=8)
    r256 = lambda x: (x + 255) // 256 * 256
    assert serve.footprint(p) == r256(workspace_bytes(p)) + r256(16 * 300 * 16) + 256
    L = _abi.lib()
    h = ctypes.c_void_p()
    good = dict(pool=ctypes.c_void_p(1 << 20), pool_bytes=1 << 20, slots=2, chunk=8, candidates=32, mode=2,
                recheck_topk=8, reserved0=0, radius0=0.05, target_factor=1.1)
    for k, v in (("pool", ctypes.c_void_p(0)), ("pool", ctypes.c_void_p((1 << 20) + 8)), ("pool_bytes", 100),
                 ("slots", 0), ("slots", 1025), ("chunk", 0), ("candidates", 0), ("radius0", 0.0)):
        bad = _abi.ServerParams(**dict(good, **{k: v}))
        assert L.trstmi_server_create(ctypes.byref(bad), ctypes.byref(h)) == _abi.E_INVALID_ARG, k
    # the engine runs the BF16-screen form only
    for mode in (0, 1):
        other = _abi.ServerParams(**dict(good, mode=mode))
        assert L.trstmi_server_create(ctypes.byref(other), ctypes.byref(h)) == _abi.E_UNSUPPORTED
    # the pool must hold the engine table first
    tb = L.trstmi_server_table_bytes(2)
    assert tb > 0 and tb % 256 == 0 and L.trstmi_server_table_bytes(0) == 0 and L.trstmi_server_table_bytes(1025) == 0
    assert L.trstmi_server_table_bytes(1024) > L.trstmi_server_table_bytes(2)
    small = _abi.ServerParams(**dict(good, pool_bytes=tb + 255))
    assert L.trstmi_server_create(ctypes.byref(small), ctypes.byref(h)) == _abi.E_INVALID_ARG
    assert L.trstmi_server_submit(None, None, None) == _abi.E_INVALID_ARG
    assert L.trstmi_server_destroy(None) == _abi.OK
    assert L.trstmi_server_forget(None, 0) == _abi.E_INVALID_ARG


def test_summary_statistics_warmup_and_empty_fields():
    """Latency = finish - arrival over finished requests, time to target over
    those that reached it; warm-up arrivals count in throughput only; an
    empty statistic is None (JSON null), never NaN."""
    R = serve.Request
    reqs = [R(id=0, arrival=0.0, n=16, d=8), R(id=1, arrival=0.1, n=16, d=8), R(id=2, arrival=0.2, n=40, d=4),
            R(id=3, arrival=0.3, n=40, d=4)]
    for r, (admit, finish, steps, reached) in zip(reqs, ((0.0, 1.0, 10, True), (0.1, 2.1, 20, False),
                                                          (0.5, 0.7, 5, True), (0.3, 4.3, 30, False))):
        r.status, r.admit, r.finish, r.steps, r.reached = "done", admit, finish, steps, reached
        r.mu = 2.0 * serve.welch_bound(r.n, r.d)
    s = serve.summarize(reqs, 10.0, 4, 0, 1, warmup=1)
    assert s["done"] == 4 and s["measured"] == 3 and s["warmup_requests"] == 1
    assert s["evals_per_s"] == (10 + 20 + 5 + 30) * 4 / 10.0            # warm-up included
    assert s["screen_tflops"] == sum(r.steps * 4 * 4.0 * r.d * r.n * (r.n - 1) for r in reqs) / 10.0 / 1e12
    assert s["reached_target"] == 1 and s["p50_time_to_target_s"] == pytest.approx(0.5)   # request 2 only
    assert s["p50_latency_s"] == pytest.approx(2.0)                       # latencies 2.0, 0.5, 4.0
    assert s["reached_by_d"] == {"8": {"done": 1, "reached_target": 0}, "4": {"done": 2, "reached_target": 1}}
    assert s["median_mu_over_welch"] == pytest.approx(2.0)
    none = serve.summarize(reqs[:1], 1.0, 4, 0, 1, warmup=1)
    assert none["p50_latency_s"] is None and none["p99_time_to_target_s"] is None and none["mean_queue_s"] is None
    assert "NaN" not in __import__("json").dumps(none)
