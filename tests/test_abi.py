"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function ``include/trstmi.h`` declares, and rejects bad arguments
before anything reaches the device."""

import ctypes
import os
import re

import pytest

from conftest import ROOT

abi = pytest.importorskip("paper_2207_06374_amd._abi")

HEADER_DIR = os.path.join(ROOT, "include")


def _declared_functions():
    names = set()
    for fn in os.listdir(HEADER_DIR):
        if fn.endswith(".h"):
            text = open(os.path.join(HEADER_DIR, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(trstmi_[a-z0-9_]+)\s*\(", text))
    return names


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(abi.LIB_PATH):
        pytest.fail("libtrstmi.so is not built (run `python -m paper_2207_06374_amd.build`)")
    return abi.lib()


def test_every_declared_symbol_is_exported(L):
    names = _declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(abi.SIGNATURES) >= names


def test_struct_sizes_match_header():
    # int64 n, d; 4 x int32; 2 x uint64; 5 doubles; int64; 2 doubles
    assert ctypes.sizeof(abi.Params) == 8 * 2 + 4 * 4 + 8 * 2 + 8 * 5 + 8 + 8 * 2
    assert ctypes.sizeof(abi.State) == 5 * 8
    assert ctypes.sizeof(abi.Report) == 4 * 8


def _params(L, n=16, d=4, **kw):
    p = abi.Params()
    L.trstmi_default_params(ctypes.byref(p), n, d)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_defaults_and_workspace(L):
    p = _params(L)
    assert p.candidates == 64 and p.mode == abi.MODE_FP64 and p.recheck_topk == 8
    assert p.radius0 == 0.1 and p.grow == 2.0 and p.shrink == 0.5 and p.radius_min == 1e-12
    assert p.radius_max == 1.0 and p.max_steps == 1000
    ws = L.trstmi_workspace_bytes(ctypes.byref(p))
    # candidate buffer: 64 candidates x 16 columns x 8 (padded 2d) doubles
    assert ws >= 64 * 16 * 8 * 8 and ws % 256 == 0
    big = _params(L, 4096, 64, candidates=128, mode=abi.MODE_BF16_SCREEN)
    assert L.trstmi_workspace_bytes(ctypes.byref(big)) >= 128 * 4096 * 128 * 2 + 8 * 4096 * 128 * 8
    assert L.trstmi_coherence_workspace_bytes(4096, 64, abi.MODE_FP64) >= 4096 * 128 * 8


@pytest.mark.parametrize("field,value", [("n", 1), ("d", 0), ("d", 513), ("candidates", 0),
                                         ("candidates", 40000), ("radius0", 0.0), ("radius0", 2.0),
                                         ("radius_min", -1.0), ("grow", 0.5), ("shrink", 0.0),
                                         ("shrink", 1.5), ("max_steps", -1), ("max_steps", 2 ** 32),
                                         ("max_steps", 10 ** 12), ("seed", 2 ** 32),
                                         ("stream_id", 2 ** 33), ("mode", 7), ("radius0", float("nan"))])
def test_invalid_params_rejected_on_host(L, field, value):
    p = _params(L, **{field: value})
    assert L.trstmi_workspace_bytes(ctypes.byref(p)) == 0
    fake = ctypes.c_void_p(256)
    st = abi.State(256, 256, 256, 256, 256)
    status = L.trstmi_step(ctypes.byref(p), ctypes.byref(st), fake, 1 << 40, None, None, None)
    assert status == abi.E_INVALID_ARG
    assert L.trstmi_last_error()


def test_step_limit_is_the_counter_word(L):
    """The step index is one 32-bit word of the random-number counter: the
    largest accepted step limit is 2^32 - 1."""
    p = _params(L, max_steps=2 ** 32 - 1)
    assert L.trstmi_workspace_bytes(ctypes.byref(p)) > 0
    p.max_steps = 2 ** 32
    assert L.trstmi_workspace_bytes(ctypes.byref(p)) == 0


def test_bf16_topk_range(L):
    p = _params(L, mode=abi.MODE_BF16_SCREEN, candidates=4, recheck_topk=5)
    assert L.trstmi_workspace_bytes(ctypes.byref(p)) == 0
    p.recheck_topk = 4
    assert L.trstmi_workspace_bytes(ctypes.byref(p)) > 0


def test_workspace_errors(L):
    p = _params(L)
    need = L.trstmi_workspace_bytes(ctypes.byref(p))
    st = abi.State(256, 256, 256, 256, 256)
    assert L.trstmi_step(ctypes.byref(p), ctypes.byref(st), None, need, None, None, None) == abi.E_WORKSPACE
    assert L.trstmi_step(ctypes.byref(p), ctypes.byref(st), ctypes.c_void_p(128), need, None, None,
                         None) == abi.E_WORKSPACE
    assert L.trstmi_step(ctypes.byref(p), ctypes.byref(st), ctypes.c_void_p(512), need - 1, None, None,
                         None) == abi.E_WORKSPACE
    assert b"workspace" in L.trstmi_last_error()


def test_state_and_pointer_errors(L):
    p = _params(L)
    st = abi.State(256, 0, 256, 256, 256)
    assert L.trstmi_init_haar(ctypes.byref(p), ctypes.byref(st), ctypes.c_void_p(256), 1 << 30,
                              None) == abi.E_INVALID_ARG
    st = abi.State(264, 256, 256, 256, 256)   # frame not 16-byte aligned
    assert L.trstmi_init_haar(ctypes.byref(p), ctypes.byref(st), ctypes.c_void_p(256), 1 << 30,
                              None) == abi.E_INVALID_ARG
    assert L.trstmi_coherence(1, 4, 0, ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256),
                              1 << 20, None) == abi.E_INVALID_ARG
    assert L.trstmi_coherence(16, 4, 9, ctypes.c_void_p(256), ctypes.c_void_p(256), ctypes.c_void_p(256),
                              1 << 20, None) == abi.E_INVALID_ARG
    assert L.trstmi_solve(ctypes.byref(p), ctypes.byref(abi.State(256, 256, 256, 256, 256)),
                          ctypes.c_void_p(256), 1 << 30, 0, None) == abi.E_INVALID_ARG
    assert L.trstmi_candidates(ctypes.byref(p), ctypes.c_void_p(256), ctypes.c_void_p(256), 0, 0, 0, None,
                               ctypes.c_void_p(256), None) == abi.E_INVALID_ARG


def test_binding_refuses_without_gpu_or_library(monkeypatch):
    """The product path has no fallback: with the library path pointing
    nowhere, loading fails loudly."""
    monkeypatch.setattr(abi, "LIB_PATH", "/nonexistent/libtrstmi.so")
    monkeypatch.setattr(abi, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        abi.lib()


def _batch(L, specs, C=8):
    inst = (abi.BatchInstance * len(specs))()
    for k, s in enumerate(specs):
        inst[k].n, inst[k].d = s[0], s[1]
        inst[k].seed, inst[k].stream_id = 0, k
        inst[k].max_steps = 10
        inst[k].waves_per_item = s[2] if len(s) > 2 else 0
    p = abi.BatchParams(len(specs), C, 0.1, 2.0, 0.5, 1e-12, 1.0, 0.0)
    return p, inst


@pytest.mark.parametrize("specs,ok", [([(16, 4)], True), ([(256, 16)], True), ([(257, 4)], False),
                                      ([(16, 17)], False), ([(1, 3)], False), ([(256, 16, 1)], False),
                                      ([(128, 16, 2)], True), ([(64, 16, 1)], True), ([(16, 4, 3)], False)])
def test_batch_validation(L, specs, ok):
    p, inst = _batch(L, specs)
    assert (L.trstmi_batch_workspace_bytes(ctypes.byref(p), inst) > 0) == ok


def test_batch_workspace_scales_with_instances(L):
    p1, i1 = _batch(L, [(16, 4)] * 4)
    p2, i2 = _batch(L, [(16, 4)] * 64)
    assert L.trstmi_batch_workspace_bytes(ctypes.byref(p2), i2) > L.trstmi_batch_workspace_bytes(ctypes.byref(p1), i1)
    p3, i3 = _batch(L, [(16, 4)], C=300)
    assert L.trstmi_batch_workspace_bytes(ctypes.byref(p3), i3) == 0


def test_round_bf16_argument_checks(L):
    assert L.trstmi_round_bf16(None, 0, None, None) == abi.OK
    assert L.trstmi_round_bf16(None, -1, None, None) == abi.E_INVALID_ARG
    assert L.trstmi_round_bf16(None, 4, ctypes.c_void_p(256), None) == abi.E_INVALID_ARG
    assert L.trstmi_round_bf16(ctypes.c_void_p(260), 4, ctypes.c_void_p(256), None) == abi.E_INVALID_ARG


def test_timing_controls_without_device(L):
    """Timing settings are host-side: enabling, limiting to one kernel and
    reading totals work (and read zero) with nothing launched."""
    assert L.trstmi_timing_only(b"gram_bf16") == abi.OK
    assert L.trstmi_timing_enable(1) == abi.OK
    assert L.trstmi_timing_enable(0) == abi.OK
    assert L.trstmi_timing_only(None) == abi.OK
    ms = ctypes.c_double(-1.0)
    cnt = ctypes.c_int64(-1)
    assert L.trstmi_timing_read(b"perturb", ctypes.byref(ms), ctypes.byref(cnt)) == abi.OK
    assert ms.value == 0.0 and cnt.value == 0
    assert L.trstmi_timing_read(None, ctypes.byref(ms), ctypes.byref(cnt)) == abi.E_INVALID_ARG
    assert L.trstmi_abi_version() >= 3


def test_lse_argument_checks(L):
    """The smooth maximum rejects bad arguments before any launch."""
    need = L.trstmi_lse_workspace_bytes(100, 8)
    assert need > 100 * 16 * 8
    assert L.trstmi_lse_workspace_bytes(1, 8) == 0 and L.trstmi_lse_workspace_bytes(100, 0) == 0
    p = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    assert L.trstmi_lse(1, 8, p, 0.1, 1, p, ws, need, None) == abi.E_INVALID_ARG          # n < 2
    assert L.trstmi_lse(100, 8, p, 0.0, 1, p, ws, need, None) == abi.E_INVALID_ARG        # delta <= 0
    assert L.trstmi_lse(100, 8, p, float("inf"), 1, p, ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_lse(100, 8, p, float("nan"), 1, p, ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_lse(100, 8, p, 0.1, 2, p, ws, need, None) == abi.E_INVALID_ARG        # squared not 0/1
    assert L.trstmi_lse(100, 8, None, 0.1, 1, p, ws, need, None) == abi.E_INVALID_ARG     # null frame
    assert L.trstmi_lse(100, 8, ctypes.c_void_p(4104), 0.1, 1, p, ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_lse(100, 8, p, 0.1, 1, p, ws, need - 1, None) == abi.E_WORKSPACE
    assert L.trstmi_abi_version() >= 4


def test_lse_grad_argument_checks(L):
    need = L.trstmi_lse_grad_workspace_bytes(100, 8)
    assert need > L.trstmi_lse_workspace_bytes(100, 8)
    assert L.trstmi_lse_grad_workspace_bytes(100, 65) == 0
    p = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    assert L.trstmi_lse_grad(100, 65, p, 0.1, p, p, ws, need, None) == abi.E_UNSUPPORTED
    assert L.trstmi_lse_grad(100, 8, p, -1.0, p, p, ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_lse_grad(100, 8, p, 0.1, p, None, ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_lse_grad(100, 8, p, 0.1, p, ctypes.c_void_p(4104), ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_lse_grad(100, 8, p, 0.1, p, p, ws, need - 1, None) == abi.E_WORKSPACE


def test_tr_step_argument_checks(L):
    need = L.trstmi_tr_workspace_bytes(100, 8)
    assert need > L.trstmi_lse_grad_workspace_bytes(100, 8)
    assert L.trstmi_tr_workspace_bytes(100, 65) == 0
    p = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    good = abi.TRParams(0.05, 0.1, 1.0, 0.1, 1e-8, 20, 1e-6)
    rep = abi.TRReport()
    assert L.trstmi_tr_step(100, 65, p, ctypes.byref(good), ctypes.byref(rep), ws, need, None) == abi.E_UNSUPPORTED
    for bad in (abi.TRParams(0.0, 0.1, 1.0, 0.1, 1e-8, 20, 1e-6), abi.TRParams(0.05, -1.0, 1.0, 0.1, 1e-8, 20, 1e-6),
                abi.TRParams(0.05, 0.1, 0.05, 0.1, 1e-8, 20, 1e-6), abi.TRParams(0.05, 0.1, 1.0, 0.3, 1e-8, 20, 1e-6),
                abi.TRParams(0.05, 0.1, 1.0, 0.1, 1e-8, 0, 1e-6), abi.TRParams(0.05, 0.1, 1.0, 0.1, 1e-8, 20, -1e-6)):
        assert L.trstmi_tr_step(100, 8, p, ctypes.byref(bad), ctypes.byref(rep), ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_tr_step(100, 8, p, None, ctypes.byref(rep), ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_tr_step(100, 8, p, ctypes.byref(good), ctypes.byref(rep), ws, need - 1, None) == abi.E_WORKSPACE


def test_lse_hvp_argument_checks(L):
    need = L.trstmi_lse_hvp_workspace_bytes(100, 8)
    assert need > L.trstmi_lse_workspace_bytes(100, 8)
    assert L.trstmi_lse_hvp_workspace_bytes(100, 65) == 0 and L.trstmi_lse_hvp_workspace_bytes(1, 8) == 0
    p = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    assert L.trstmi_lse_hvp(100, 65, p, p, 0.1, p, p, ws, need, None) == abi.E_UNSUPPORTED
    assert L.trstmi_lse_hvp(100, 8, p, p, 0.0, p, p, ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_lse_hvp(100, 8, p, None, 0.1, p, p, ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_lse_hvp(100, 8, p, ctypes.c_void_p(4104), 0.1, p, p, ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_lse_hvp(100, 8, p, p, 0.1, p, p, ws, need - 1, None) == abi.E_WORKSPACE
    assert L.trstmi_abi_version() >= 11


def test_coherence_noalloc_refuses_oversized_frames_on_the_host(L):
    """The fixed workspace bounds the frame; a larger one is refused before
    any device call (this runs without a GPU)."""
    cap = L.trstmi_coherence_noalloc_max_bytes()
    assert cap == (16 << 20) + 256
    p = ctypes.c_void_p(4096)
    n_big = cap // (1024 * 8) + 1
    assert L.trstmi_coherence_noalloc(n_big, 512, 0, p, p, None) == abi.E_UNSUPPORTED
    assert b"fixed workspace" in L.trstmi_last_error()
    assert L.trstmi_coherence_workspace_bytes(n_big - 1, 512, 0) <= cap
    assert L.trstmi_coherence_noalloc(1, 4, 0, p, p, None) == abi.E_INVALID_ARG
    assert L.trstmi_coherence_noalloc(16, 4, 7, p, p, None) == abi.E_INVALID_ARG


def test_screen_tiles_argument_checks(L):
    T = abi.ScreenTile
    good = (T * 2)(T(4, 512, 0, 6), T(8, 1024, 1, 64))
    assert L.trstmi_screen_tiles_set(good, 2) == abi.OK
    for bad in (T(0, 512, 0, 6), T(9, 512, 1, 6), T(4, 1, 0, 6), T(4, 512, 2, 6), T(5, 512, 0, 6),
                T(4, 512, 0, 0), T(4, 512, 1, 65)):
        one = (T * 1)(bad)
        assert L.trstmi_screen_tiles_set(one, 1) == abi.E_INVALID_ARG
    assert L.trstmi_screen_tiles_set(None, 1) == abi.E_INVALID_ARG
    assert L.trstmi_screen_tiles_set(None, -1) == abi.E_INVALID_ARG
    assert L.trstmi_screen_tiles_set(None, 0) == abi.OK
    abi._install_screen_tiles(L)
    assert L.trstmi_abi_version() >= 12


def test_optimize_batched_argument_checks(L):
    assert L.trstmi_optimize_batched_workspace_bytes(129, 4, 8) == 0
    assert L.trstmi_optimize_batched_workspace_bytes(64, 17, 8) == 0
    assert L.trstmi_optimize_batched_workspace_bytes(64, 4, 0) == 0
    need = L.trstmi_optimize_batched_workspace_bytes(16, 4, 8)
    assert need >= 8 * 10 * 2 * 4 * 16 * 8
    dl = (ctypes.c_double * 2)(0.1, 0.01)
    mu = ctypes.c_double()
    best = ctypes.c_int32()
    p = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    good = abi.OptParams(0, 8, 2, dl, 10, 0.1, 1e-10, 1.0, 0.1, 1e-10, 0, 0.0, 1, 0)
    assert L.trstmi_optimize_batched(200, 4, ctypes.byref(good), p, ctypes.byref(mu), ctypes.byref(best), ws, need,
                                     None) == abi.E_UNSUPPORTED
    fd = abi.OptParams(0, 8, 2, dl, 10, 0.1, 1e-10, 1.0, 0.1, 1e-10, 0, 1e-6, 1, 0)
    assert L.trstmi_optimize_batched(16, 4, ctypes.byref(fd), p, ctypes.byref(mu), ctypes.byref(best), ws, need,
                                     None) == abi.E_UNSUPPORTED
    bad = abi.OptParams(0, 8, 2, dl, 0, 0.1, 1e-10, 1.0, 0.1, 1e-10, 0, 0.0, 1, 0)
    assert L.trstmi_optimize_batched(16, 4, ctypes.byref(bad), p, ctypes.byref(mu), ctypes.byref(best), ws, need,
                                     None) == abi.E_INVALID_ARG
    assert L.trstmi_optimize_batched(16, 4, ctypes.byref(good), p, ctypes.byref(mu), ctypes.byref(best), ws,
                                     need - 1, None) == abi.E_WORKSPACE
    assert L.trstmi_abi_version() >= 13


def test_optimize_argument_checks(L):
    need = L.trstmi_optimize_workspace_bytes(9, 3, 1)
    assert need > L.trstmi_tr_workspace_bytes(9, 3)
    assert L.trstmi_optimize_workspace_bytes(9, 65, 1) == 0
    assert L.trstmi_optimize_workspace_bytes(9, 3, 0) == 0 and L.trstmi_optimize_workspace_bytes(9, 3, 65) == 0
    assert L.trstmi_optimize_workspace_bytes(9, 3, 4) == 4 * need
    dl = (ctypes.c_double * 2)(0.1, 0.01)
    mu = ctypes.c_double()
    best = ctypes.c_int32()
    p = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    good = abi.OptParams(0, 2, 2, dl, 10, 0.1, 1e-10, 1.0, 0.1, 1e-10, 0, 1e-6, 1, 0)
    assert L.trstmi_optimize(9, 65, ctypes.byref(good), p, ctypes.byref(mu), ctypes.byref(best), ws, need,
                             None) == abi.E_UNSUPPORTED
    bad_dl = (ctypes.c_double * 2)(0.1, -1.0)
    for bad in (abi.OptParams(0, 0, 2, dl, 10, 0.1, 1e-10, 1.0, 0.1, 1e-10, 0, 1e-6, 1, 0),
                abi.OptParams(0, 2, 2, bad_dl, 10, 0.1, 1e-10, 1.0, 0.1, 1e-10, 0, 1e-6, 1, 0),
                abi.OptParams(0, 2, 2, dl, 0, 0.1, 1e-10, 1.0, 0.1, 1e-10, 0, 1e-6, 1, 0),
                abi.OptParams(0, 2, 2, dl, 10, 0.1, 1e-10, 0.01, 0.1, 1e-10, 0, 1e-6, 1, 0),
                abi.OptParams(0, 2, 2, dl, 10, 0.1, 1e-10, 1.0, 0.1, 1e-10, 0, 1e-6, 0, 0),
                abi.OptParams(0, 2, 2, dl, 10, 0.1, 1e-10, 1.0, 0.1, 1e-10, 0, 1e-6, 65, 0),
                abi.OptParams(0, 2, 2, dl, 10, 0.1, 1e-10, 1.0, 0.1, 1e-10, 0, -1e-6, 1, 0),
                abi.OptParams(0, 2, 2, dl, 10, 0.1, 1e-10, 1.0, 0.1, 1e-10, 0, 1e-6, 1, -1)):
        assert L.trstmi_optimize(9, 3, ctypes.byref(bad), p, ctypes.byref(mu), ctypes.byref(best), ws, need,
                                 None) == abi.E_INVALID_ARG
    assert L.trstmi_optimize(9, 3, ctypes.byref(good), p, None, ctypes.byref(best), ws, need,
                             None) == abi.E_INVALID_ARG
    assert L.trstmi_optimize(9, 3, ctypes.byref(good), p, ctypes.byref(mu), ctypes.byref(best), ws, need - 1,
                             None) == abi.E_WORKSPACE
    four = abi.OptParams(0, 8, 2, dl, 10, 0.1, 1e-10, 1.0, 0.1, 1e-10, 0, 1e-6, 4, 0)
    assert L.trstmi_optimize(9, 3, ctypes.byref(four), p, ctypes.byref(mu), ctypes.byref(best), ws, 4 * need - 1,
                             None) == abi.E_WORKSPACE
    assert L.trstmi_abi_version() >= 9


def test_miso_argument_checks(L):
    """The codebook quantiser rejects bad arguments before any launch."""
    need = L.trstmi_miso_workspace_bytes(100, 8, 1000)
    assert need >= 100 * 16 * 8 + 16 * 16
    assert L.trstmi_miso_workspace_bytes(0, 8, 10) == 0 and L.trstmi_miso_workspace_bytes(10, 0, 10) == 0
    assert L.trstmi_miso_workspace_bytes(10, 8, -1) == 0 and L.trstmi_miso_workspace_bytes(10, 513, 10) == 0
    assert L.trstmi_miso_workspace_bytes(1, 1, 0) > 0
    p = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    args = lambda **k: dict(dict(cb=p, n=100, d=8, ch=p, m=1000, idx=p, g=p, dist=p, s=p, ws=ws, wsb=need), **k)

    def call(**k):
        a = args(**k)
        return L.trstmi_miso_quantize(a["cb"], a["n"], a["d"], a["ch"], a["m"], a["idx"], a["g"], a["dist"], a["s"],
                                      a["ws"], a["wsb"], None)

    assert call(n=0) == abi.E_INVALID_ARG
    assert call(n=(1 << 18) + 1) == abi.E_INVALID_ARG
    assert call(d=0) == abi.E_INVALID_ARG and call(d=513) == abi.E_INVALID_ARG
    assert call(m=-1) == abi.E_INVALID_ARG and call(m=1 << 31) == abi.E_INVALID_ARG
    assert call(cb=None) == abi.E_INVALID_ARG
    assert call(ch=None) == abi.E_INVALID_ARG
    assert call(ch=ctypes.c_void_p(4104)) == abi.E_INVALID_ARG
    assert call(idx=ctypes.c_void_p(4098)) == abi.E_INVALID_ARG
    assert call(s=ctypes.c_void_p(4100)) == abi.E_INVALID_ARG
    assert call(wsb=need - 1) == abi.E_WORKSPACE
    assert call(ws=None) == abi.E_WORKSPACE
    assert L.trstmi_abi_version() >= 5


def test_coherence_pair_and_shutdown_without_device(L):
    need = L.trstmi_coherence_workspace_bytes(100, 8, abi.MODE_FP64)
    p = ctypes.c_void_p(4096)
    ws = ctypes.c_void_p(1 << 20)
    assert L.trstmi_coherence_pair(1, 8, p, p, p, ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_coherence_pair(100, 8, None, p, p, ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_coherence_pair(100, 8, p, p, None, ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_coherence_pair(100, 8, p, p, ctypes.c_void_p(4100), ws, need, None) == abi.E_INVALID_ARG
    assert L.trstmi_coherence_pair(100, 8, p, p, p, ws, need - 1, None) == abi.E_WORKSPACE
    assert L.trstmi_shutdown() == abi.OK
    assert L.trstmi_abi_version() >= 7


def test_c_abi_from_plain_c():
    """A C11 program includes the header, links the library and calls the
    host-side entry points (no GPU needed)."""
    import os
    import shutil
    import subprocess
    import tempfile
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    pkg = os.path.join(root, "paper_2207_06374_amd")
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "c_abi_check")
        subprocess.run(["gcc", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(root, "include"),
                        "-I", "/opt/rocm/include", os.path.join(root, "tests", "c_abi_check.c"), "-o", exe,
                        "-L", pkg, "-ltrstmi", "-Wl,-rpath," + pkg], check=True, capture_output=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
        assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stdout, r.stderr)


def test_screen_bounds_equal_the_oracle(L):
    """The bounds the library prunes its FP64 rechecks with are the oracle's
    pinned ones (two independent writings of the same formulas)."""
    import math

    import oracle
    assert L.trstmi_abi_version() >= 14
    for d in (1, 2, 3, 7, 16, 33, 64, 128, 512):
        assert L.trstmi_bf16_screen_bound(d) == pytest.approx(oracle.screen_error_bound(d), rel=1e-14, abs=0)
    for d in range(1, 17):
        assert L.trstmi_batch_screen_bound(d) == pytest.approx(oracle.split_screen_error_bound(d), rel=1e-14, abs=0)
    assert math.isnan(L.trstmi_bf16_screen_bound(0))
    assert math.isnan(L.trstmi_batch_screen_bound(0)) and math.isnan(L.trstmi_batch_screen_bound(17))


def test_autotuner_feasibility_matches_the_library(L):
    """The autotuner's copy of the batched kernel's LDS rule (which
    waves_per_item values fit an instance) agrees with the library's own
    host check for every d <= 16 and every N the batched form takes."""
    autotune = pytest.importorskip("paper_2207_06374_amd.autotune")
    for d in range(1, 17):
        for n in sorted({2, 3, d + 1, 17, 32, 33, 64, 65, 82, 83, 100, 115, 116, 128, 129, 164, 165, 192, 230, 255, 256}):
            if n > 256:
                continue
            feasible = autotune.feasible(n, d)
            for w in (1, 2, 4):
                p, inst = _batch(L, [(n, d, w)])
                assert (L.trstmi_batch_workspace_bytes(ctypes.byref(p), inst) > 0) == (w in feasible), (n, d, w)
