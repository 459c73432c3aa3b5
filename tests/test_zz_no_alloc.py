"""GPU check of trstmi_coherence_noalloc (the entry point for callers that
cannot allocate): through the C ABI, its result equals trstmi_coherence's
with a caller workspace, bit for bit, on two calls in a row with the second
smaller than the first, in every mode; a frame above the fixed workspace is
refused before anything runs."""

import ctypes

import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lib = pytest.importorskip("paper_2207_06374_amd")
abi = lib._abi


def _noalloc(dev, n, d, mode):
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    st = abi.lib().trstmi_coherence_noalloc(n, d, mode, dev.data_ptr(), out.data_ptr(), None)
    assert st == abi.OK, abi.lib().trstmi_last_error()
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("mode", [lib.MODE_FP64, lib.MODE_FP32, lib.MODE_BF16_SCREEN])
def test_noalloc_equals_workspace_call_twice_shrinking(mode):
    for n, d, seed in ((1500, 48, 1), (300, 7, 2)):   # second call smaller: stale scratch must not leak in
        Y = inputs.random_frame(n, d, seed=seed)
        dev = lib.frame_to_device(Y)
        print(f"mode={mode} n={n} d={d}", flush=True)
        got = _noalloc(dev, n, d, mode)
        want = lib.coherence(dev, n, d, mode=mode)
        torch.cuda.synchronize()
        assert torch.equal(got, want), (got.item(), want.item())
        if mode == lib.MODE_FP64:
            import oracle
            assert abs(got.item() - oracle.coherence(Y)) <= 1e-12


def test_noalloc_zero_column_and_limit():
    n, d = 40, 5
    Y = inputs.random_frame(n, d, seed=3)
    Y[:, 7] = 0
    got = _noalloc(lib.frame_to_device(Y), n, d, lib.MODE_FP64)
    assert got.item() == float("inf")
    cap = abi.lib().trstmi_coherence_noalloc_max_bytes()
    # n * ld * 8 bytes must fit: ld = 2d rounded up to 8 -> d = 512 gives ld = 1024
    n_big = cap // (1024 * 8) + 1
    out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    frame = torch.ones(2 * 512 * int(n_big), dtype=torch.float64, device="cuda")   # a valid frame: refused for size
    st = abi.lib().trstmi_coherence_noalloc(int(n_big), 512, lib.MODE_FP64, frame.data_ptr(), out.data_ptr(), None)
    assert st == abi.E_UNSUPPORTED
    assert b"fixed workspace" in abi.lib().trstmi_last_error()
    torch.cuda.synchronize()
    assert out.item() == -1.0
