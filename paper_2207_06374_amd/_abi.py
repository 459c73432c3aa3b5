"""ctypes declarations of the C ABI in ``include/trstmi.h`` (marshalling only).

The shared library is built in-tree (``paper_2207_06374_amd/libtrstmi.so``).
There is no fallback: if the library is missing, loading raises.
"""

from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtrstmi.so")

OK = 0
E_INVALID_ARG = 1
E_WORKSPACE = 2
E_HIP = 3
E_UNSUPPORTED = 4

MODE_FP64 = 0
MODE_FP32 = 1
MODE_BF16_SCREEN = 2

FLAG_ACCEPTED = 1
FLAG_DONE = 2
FLAG_NEAR_TIE = 4
FLAG_NO_VALID = 8

MAX_D = 512
MAX_CANDIDATES = 32768
MAX_TOPK = 64


class Params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("d", ctypes.c_int64),
        ("candidates", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("recheck_topk", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("stream_id", ctypes.c_uint64),
        ("radius0", ctypes.c_double),
        ("grow", ctypes.c_double),
        ("shrink", ctypes.c_double),
        ("radius_min", ctypes.c_double),
        ("radius_max", ctypes.c_double),
        ("max_steps", ctypes.c_int64),
        ("target_mu", ctypes.c_double),
        ("near_tie", ctypes.c_double),
    ]


class State(ctypes.Structure):
    _fields_ = [
        ("frame", ctypes.c_void_p),
        ("mu", ctypes.c_void_p),
        ("radius", ctypes.c_void_p),
        ("step", ctypes.c_void_p),
        ("flags", ctypes.c_void_p),
    ]


class Report(ctypes.Structure):
    _fields_ = [
        ("cand_mu", ctypes.c_void_p),
        ("rechecked", ctypes.c_void_p),
        ("recheck_mu", ctypes.c_void_p),
        ("best", ctypes.c_void_p),
    ]


class BatchInstance(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("d", ctypes.c_int32),
        ("seed", ctypes.c_uint32),
        ("stream_id", ctypes.c_uint32),
        ("target_mu", ctypes.c_double),
        ("max_steps", ctypes.c_int64),
        ("waves_per_item", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class BatchParams(ctypes.Structure):
    _fields_ = [
        ("count", ctypes.c_int32),
        ("candidates", ctypes.c_int32),
        ("radius0", ctypes.c_double),
        ("grow", ctypes.c_double),
        ("shrink", ctypes.c_double),
        ("radius_min", ctypes.c_double),
        ("radius_max", ctypes.c_double),
        ("near_tie", ctypes.c_double),
    ]


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_sz = ctypes.c_size_t

class TRParams(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("radius", ctypes.c_double), ("radius_max", ctypes.c_double),
                ("eta", ctypes.c_double), ("cg_tol", ctypes.c_double), ("cg_max_iter", ctypes.c_int32),
                ("fd_step", ctypes.c_double)]


class OptParams(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("restarts", ctypes.c_int32), ("n_deltas", ctypes.c_int32),
                ("deltas", ctypes.POINTER(ctypes.c_double)), ("steps_per_delta", ctypes.c_int32),
                ("radius0", ctypes.c_double), ("radius_min", ctypes.c_double), ("radius_max", ctypes.c_double),
                ("eta", ctypes.c_double), ("cg_tol", ctypes.c_double), ("cg_max_iter", ctypes.c_int32),
                ("fd_step", ctypes.c_double), ("concurrency", ctypes.c_int32), ("first_restart", ctypes.c_int32)]


class TRReport(ctypes.Structure):
    _fields_ = [("f_old", ctypes.c_double), ("f_new", ctypes.c_double), ("rho", ctypes.c_double),
                ("step_norm", ctypes.c_double), ("new_radius", ctypes.c_double), ("cg_iters", ctypes.c_int32),
                ("cg_exit", ctypes.c_int32), ("accepted", ctypes.c_int32)]


class ServerParams(ctypes.Structure):
    _fields_ = [("pool", ctypes.c_void_p), ("pool_bytes", ctypes.c_uint64), ("slots", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("candidates", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("recheck_topk", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("radius0", ctypes.c_double),
                ("target_factor", ctypes.c_double)]


class ServeRequest(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int64), ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint64),
                ("target_mu", ctypes.c_double), ("max_steps", ctypes.c_int64)]


class RequestResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reached", ctypes.c_int32), ("mu", ctypes.c_double),
                ("steps", ctypes.c_int64), ("target_mu", ctypes.c_double), ("queue_s", ctypes.c_double),
                ("run_s", ctypes.c_double), ("footprint", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("pool_capacity", ctypes.c_uint64), ("pool_used", ctypes.c_uint64), ("pool_peak", ctypes.c_uint64),
                ("active", ctypes.c_int32), ("queued", ctypes.c_int32), ("submitted", ctypes.c_int64)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_ERROR, REQ_REJECTED, REQ_CANCELLED = range(6)


# name: (restype, argtypes)
SIGNATURES = {
    "trstmi_default_params": (None, [_P(Params), _i64, _i64]),
    "trstmi_workspace_bytes": (_sz, [_P(Params)]),
    "trstmi_coherence_workspace_bytes": (_sz, [_i64, _i64, _i32]),
    "trstmi_coherence": (_i32, [_i64, _i64, _i32, _vp, _vp, _vp, _sz, _vp]),
    "trstmi_coherence_pair": (_i32, [_i64, _i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "trstmi_lse_workspace_bytes": (_sz, [_i64, _i64]),
    "trstmi_lse": (_i32, [_i64, _i64, _vp, ctypes.c_double, _i32, _vp, _vp, _sz, _vp]),
    "trstmi_lse_grad_workspace_bytes": (_sz, [_i64, _i64]),
    "trstmi_lse_grad": (_i32, [_i64, _i64, _vp, ctypes.c_double, _vp, _vp, _vp, _sz, _vp]),
    "trstmi_server_table_bytes": (_sz, [_i32]),
    "trstmi_screen_tiles_set": (_i32, [_vp, _i32]),
    "trstmi_optimize_batched_workspace_bytes": (_sz, [_i64, _i64, _i32]),
    "trstmi_optimize_batched": (_i32, [_i64, _i64, _P(OptParams), _vp, _P(ctypes.c_double), _P(ctypes.c_int32), _vp,
                                       _sz, _vp]),
    "trstmi_welch_bound": (ctypes.c_double, [_i64, _i64]),
    "trstmi_bf16_screen_bound": (ctypes.c_double, [_i64]),
    "trstmi_batch_screen_bound": (ctypes.c_double, [ctypes.c_int32]),
    "trstmi_coherence_noalloc_max_bytes": (_sz, []),
    "trstmi_coherence_noalloc": (_i32, [_i64, _i64, _i32, _vp, _vp, _vp]),
    "trstmi_lse_hvp_workspace_bytes": (_sz, [_i64, _i64]),
    "trstmi_lse_hvp": (_i32, [_i64, _i64, _vp, _vp, ctypes.c_double, _vp, _vp, _vp, _sz, _vp]),
    "trstmi_tr_workspace_bytes": (_sz, [_i64, _i64]),
    "trstmi_tr_step": (_i32, [_i64, _i64, _vp, _P(TRParams), _P(TRReport), _vp, _sz, _vp]),
    "trstmi_optimize_workspace_bytes": (_sz, [_i64, _i64, _i32]),
    "trstmi_optimize": (_i32, [_i64, _i64, _P(OptParams), _vp, _P(ctypes.c_double), _P(_i32), _vp, _sz, _vp]),
    "trstmi_miso_workspace_bytes": (_sz, [_i64, _i64, _i64]),
    "trstmi_miso_quantize": (_i32, [_vp, _i64, _i64, _vp, _i64, _vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "trstmi_init_haar": (_i32, [_P(Params), _P(State), _vp, _sz, _vp]),
    "trstmi_candidates": (_i32, [_P(Params), _vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp]),
    "trstmi_step": (_i32, [_P(Params), _P(State), _vp, _sz, _vp, _P(Report), _vp]),
    "trstmi_solve": (_i32, [_P(Params), _P(State), _vp, _sz, _i32, _vp]),
    "trstmi_batch_workspace_bytes": (_sz, [_P(BatchParams), _P(BatchInstance)]),
    "trstmi_batch_init": (_i32, [_P(BatchParams), _P(BatchInstance), _vp, _sz, _vp]),
    "trstmi_batch_step": (_i32, [_P(BatchParams), _P(BatchInstance), _vp, _sz, _i32, _vp, _vp, _vp]),
    "trstmi_batch_run": (_i32, [_P(BatchParams), _P(BatchInstance), _vp, _sz, _i32, _i64, _P(_i32), _vp]),
    "trstmi_batch_query": (_i32, [_P(BatchParams), _P(BatchInstance), _vp, _sz, _vp, _vp, _vp, _vp, _P(_i32),
                                  _vp]),
    "trstmi_batch_frame": (_i32, [_P(BatchParams), _P(BatchInstance), _vp, _sz, _i32, _vp, _vp]),
    "trstmi_round_bf16": (_i32, [_vp, _i64, _vp, _vp]),
    "trstmi_timing_enable": (_i32, [_i32]),
    "trstmi_timing_only": (_i32, [ctypes.c_char_p]),
    "trstmi_timing_reset": (_i32, []),
    "trstmi_timing_read": (_i32, [ctypes.c_char_p, _P(ctypes.c_double), _P(_i64)]),
    "trstmi_last_error": (ctypes.c_char_p, []),
    "trstmi_request_footprint": (_sz, [_P(Params)]),
    "trstmi_server_create": (_i32, [_P(ServerParams), _P(ctypes.c_void_p)]),
    "trstmi_server_submit": (_i32, [_vp, _P(ServeRequest), _P(_i64)]),
    "trstmi_server_poll": (_i32, [_vp, _i64, _P(RequestResult)]),
    "trstmi_server_wait": (_i32, [_vp, _i64, ctypes.c_double, _P(RequestResult)]),
    "trstmi_server_cancel": (_i32, [_vp, _i64]),
    "trstmi_server_forget": (_i32, [_vp, _i64]),
    "trstmi_server_get_stats": (_i32, [_vp, _P(ServerStats)]),
    "trstmi_server_destroy": (_i32, [_vp]),
    "trstmi_shutdown": (_i32, []),
    "trstmi_abi_version": (_i32, []),
}

_lib = None


def lib():
    """The loaded library (loaded once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2207_06374_amd.build` "
                "(there is no non-HIP implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        _install_screen_tiles(L)
    return _lib


class ScreenTile(ctypes.Structure):
    _fields_ = [("ks", _i32), ("n_max", _i32), ("form", _i32), ("seg", _i32)]


SCREEN_TILES_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "screen_tiles.json")


def set_screen_tiles(entries, L=None):
    """Installs a BF16 screen tile table: a list of dicts with ks, n_max,
    form and seg (an empty list restores the library's defaults)."""
    L = L or lib()
    arr = (ScreenTile * max(len(entries), 1))(*[ScreenTile(int(e["ks"]), int(e["n_max"]), int(e["form"]),
                                                             int(e["seg"])) for e in entries])
    check(L.trstmi_screen_tiles_set(arr, len(entries)), "trstmi_screen_tiles_set")


def _install_screen_tiles(L):
    """The tuned table shipped with the package (written by autotune), if any."""
    import json
    if os.path.exists(SCREEN_TILES_PATH):
        with open(SCREEN_TILES_PATH) as f:
            set_screen_tiles(json.load(f).get("entries", []), L)


class TrstmiError(RuntimeError):
    def __init__(self, status, where):
        msg = lib().trstmi_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


def check(status, where):
    if status != OK:
        raise TrstmiError(status, where)
    return status
