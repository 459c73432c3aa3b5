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
