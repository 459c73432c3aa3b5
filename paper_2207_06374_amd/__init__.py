"""Python binding of the MI355X candidate-coherence library (libtrstmi.so).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory and streams.  The entry points have
the names of the C ABI (``include/trstmi.h``) without the ``trstmi_`` prefix:
``coherence``, ``init_haar``, ``candidates``, ``step``, ``solve``,
``workspace_bytes``, ``default_params``.  ``Solver`` bundles a state and a
workspace for one search.

Frame layout on the device: 2*d*N doubles, column-major, interleaved
(re, im).  ``frame_to_device`` / ``frame_from_device`` convert from / to a
numpy (d, N) complex128 array.
"""

from __future__ import annotations

import ctypes
import dataclasses

import numpy as np

from . import _abi
from ._abi import (  # noqa: F401
    FLAG_ACCEPTED,
    FLAG_DONE,
    FLAG_NEAR_TIE,
    FLAG_NO_VALID,
    MODE_BF16_SCREEN,
    MODE_FP32,
    MODE_FP64,
    TrstmiError,
)

MODES = {"fp64": MODE_FP64, "fp32": MODE_FP32, "bf16": MODE_BF16_SCREEN}


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2207_06374_amd needs a ROCm GPU (torch.cuda is not available)")
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def default_params(n, d, **kw):
    """A ``Params`` struct with the library defaults, overridden by ``kw``
    (``mode`` may be 'fp64' / 'fp32' / 'bf16' or the integer code)."""
    p = _abi.Params()
    _abi.lib().trstmi_default_params(ctypes.byref(p), int(n), int(d))
    for k, v in kw.items():
        if k == "mode" and isinstance(v, str):
            v = MODES[v]
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def workspace_bytes(params):
    nbytes = _abi.lib().trstmi_workspace_bytes(ctypes.byref(params))
    if nbytes == 0:
        raise _abi.TrstmiError(_abi.E_INVALID_ARG, "workspace_bytes")
    return nbytes


def coherence_workspace_bytes(n, d, mode):
    return _abi.lib().trstmi_coherence_workspace_bytes(int(n), int(d), int(mode))


def frame_to_device(F, device="cuda"):
    """numpy (d, N) complex -> flat float64 device tensor in the library layout."""
    torch = _torch()
    F = np.asarray(F, dtype=np.complex128)
    flat = np.ascontiguousarray(F.T).view(np.float64).ravel()
    return torch.from_numpy(flat.copy()).to(device)


def frame_from_device(t, n, d):
    """Flat float64 tensor in the library layout -> numpy (d, N) complex128."""
    a = t.detach().to("cpu").numpy().reshape(int(n), int(d), 2)
    return (a[..., 0] + 1j * a[..., 1]).T.copy()


def coherence(frame, n, d, mode=MODE_FP64, mu_out=None, workspace=None, stream=None):
    """Coherence of a device frame (flat float64 tensor).  Returns the device
    tensor holding mu (shape (1,), float64)."""
    torch = _torch()
    mode = MODES.get(mode, mode)
    if mu_out is None:
        mu_out = torch.empty(1, dtype=torch.float64, device=frame.device)
    need = coherence_workspace_bytes(n, d, mode)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=frame.device)
    _abi.check(_abi.lib().trstmi_coherence(int(n), int(d), int(mode), _ptr(frame), _ptr(mu_out),
                                           _ptr(workspace), workspace.numel(), _stream(stream)),
               "trstmi_coherence")
    return mu_out


def coherence_pair(frame, n, d, workspace=None, stream=None):
    """FP64 coherence of a device frame and a pair (j, k), j < k, attaining
    it (the first in the order j * n + k).  Returns device tensors (mu of
    shape (1,), pair int64 of shape (2,))."""
    torch = _torch()
    mu = torch.empty(1, dtype=torch.float64, device=frame.device)
    pair = torch.empty(2, dtype=torch.int64, device=frame.device)
    if workspace is None:
        need = _abi.lib().trstmi_coherence_workspace_bytes(int(n), int(d), MODE_FP64)
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=frame.device)
    _abi.check(_abi.lib().trstmi_coherence_pair(int(n), int(d), _ptr(frame), _ptr(mu), _ptr(pair), _ptr(workspace),
                                                workspace.numel(), _stream(stream)), "trstmi_coherence_pair")
    return mu, pair


def shutdown():
    """Release the library's internal state (pooled timing events)."""
    _abi.check(_abi.lib().trstmi_shutdown(), "trstmi_shutdown")


def lse_workspace_bytes(n, d):
    return _abi.lib().trstmi_lse_workspace_bytes(int(n), int(d))


def lse(frame, n, d, delta, squared=True, out=None, workspace=None, stream=None):
    """Smooth maximum of a device frame: (s, F) with x = |G_jk|^2 (or |G_jk|),
    j < k, s = max x and F = s + delta log sum exp((x - s) / delta), FP64.
    Returns the device tensor (shape (2,), float64)."""
    torch = _torch()
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=frame.device)
    need = lse_workspace_bytes(n, d)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=frame.device)
    _abi.check(_abi.lib().trstmi_lse(int(n), int(d), _ptr(frame), float(delta), 1 if squared else 0, _ptr(out),
                                     _ptr(workspace), workspace.numel(), _stream(stream)), "trstmi_lse")
    return out


def lse_grad_workspace_bytes(n, d):
    return _abi.lib().trstmi_lse_grad_workspace_bytes(int(n), int(d))


def lse_grad(frame, n, d, delta, out=None, grad=None, workspace=None, stream=None):
    """Smooth maximum over |G_jk|^2 and its gradient with respect to the
    (unnormalised) device frame.  Returns (out, grad): out = (s, F) (shape
    (2,), float64); grad has the frame's layout, dF = sum Re(conj(g) dframe)."""
    torch = _torch()
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=frame.device)
    if grad is None:
        grad = torch.empty_like(frame)
    need = lse_grad_workspace_bytes(n, d)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=frame.device)
    _abi.check(_abi.lib().trstmi_lse_grad(int(n), int(d), _ptr(frame), float(delta), _ptr(out), _ptr(grad),
                                          _ptr(workspace), workspace.numel(), _stream(stream)), "trstmi_lse_grad")
    return out, grad


def lse_hvp_workspace_bytes(n, d):
    return _abi.lib().trstmi_lse_hvp_workspace_bytes(int(n), int(d))


def lse_hvp(frame, v, n, d, delta, out=None, hv=None, workspace=None, stream=None):
    """Exact Hessian-vector product of the smooth maximum over |G_jk|^2 at
    the (unnormalised) device frame along the device direction v (frame
    layout).  Returns (out, hv): out = (s, F); hv has the frame's layout."""
    torch = _torch()
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=frame.device)
    if hv is None:
        hv = torch.empty_like(frame)
    need = lse_hvp_workspace_bytes(n, d)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=frame.device)
    _abi.check(_abi.lib().trstmi_lse_hvp(int(n), int(d), _ptr(frame), _ptr(v), float(delta), _ptr(out), _ptr(hv),
                                         _ptr(workspace), workspace.numel(), _stream(stream)), "trstmi_lse_hvp")
    return out, hv


def tr_workspace_bytes(n, d):
    return _abi.lib().trstmi_tr_workspace_bytes(int(n), int(d))


def tr_step(frame, n, d, delta, radius, radius_max=1.0, eta=0.1, cg_tol=1e-8, cg_max_iter=20, fd_step=0.0,
            workspace=None, stream=None):
    """One trust-region step (Steihaug CG + ratio test) on the smooth maximum
    of the device frame, updated in place when the step is taken.  fd_step 0
    uses exact Hessian-vector products, fd_step > 0 central differences of
    the gradient.  Returns the report as a dict."""
    torch = _torch()
    p = _abi.TRParams(float(delta), float(radius), float(radius_max), float(eta), float(cg_tol), int(cg_max_iter),
                      float(fd_step))
    rep = _abi.TRReport()
    if workspace is None:
        workspace = torch.empty(max(tr_workspace_bytes(n, d), 1), dtype=torch.uint8, device=frame.device)
    _abi.check(_abi.lib().trstmi_tr_step(int(n), int(d), _ptr(frame), ctypes.byref(p), ctypes.byref(rep),
                                         _ptr(workspace), workspace.numel(), _stream(stream)), "trstmi_tr_step")
    return {k: getattr(rep, k) for k, _ in _abi.TRReport._fields_}


def optimize(n, d, restarts=None, deltas=(1e-1, 3e-2, 1e-2, 3e-3, 1e-3, 3e-4, 1e-4), steps_per_delta=40, seed=0,
             radius0=0.1, radius_min=1e-10, radius_max=1.0, eta=0.1, cg_tol=1e-10, cg_max_iter=0, fd_step=0.0,
             concurrency=None, first_restart=0, device="cuda", workspace=None, stream=None, engine=None):
    """The outer procedure of Alg. 2 (delta continuation and random restarts
    around trust-region steps).  Returns (best frame as a device tensor,
    best coherence, best restart index).  restarts defaults to 2 d^2.  The
    starts are first_restart .. first_restart + restarts - 1, so one run may
    be split into calls.  engine "batched": every start in one block of a
    single launch (n <= 128, d <= 16, exact Hessian products); "threads":
    concurrency starts in flight on host threads with a stream each
    (default min(restarts, 16)), host-driven steps; None: "batched" where it
    applies."""
    torch = _torch()
    L = int(restarts) if restarts is not None else 2 * int(d) * int(d)
    P = int(concurrency) if concurrency is not None else min(L, 16)
    if engine is None:
        engine = "batched" if int(n) <= 128 and int(d) <= 16 and float(fd_step) == 0.0 else "threads"
    dl = (ctypes.c_double * len(deltas))(*[float(x) for x in deltas])
    p = _abi.OptParams(int(seed), L, len(deltas), dl, int(steps_per_delta), float(radius0), float(radius_min),
                       float(radius_max), float(eta), float(cg_tol), int(cg_max_iter), float(fd_step), P,
                       int(first_restart))
    out = torch.empty(2 * int(d) * int(n), dtype=torch.float64, device=device)
    if engine == "batched":
        if workspace is None:
            need = _abi.lib().trstmi_optimize_batched_workspace_bytes(int(n), int(d), L)
            workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=device)
        mu = ctypes.c_double()
        best = ctypes.c_int32()
        _abi.check(_abi.lib().trstmi_optimize_batched(int(n), int(d), ctypes.byref(p), _ptr(out), ctypes.byref(mu),
                                                      ctypes.byref(best), _ptr(workspace), workspace.numel(),
                                                      _stream(stream)), "trstmi_optimize_batched")
        return out, mu.value, best.value
    if engine != "threads":
        raise ValueError("engine must be None, 'batched' or 'threads'")
    if workspace is None:
        need = _abi.lib().trstmi_optimize_workspace_bytes(int(n), int(d), P)
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=device)
    mu = ctypes.c_double()
    best = ctypes.c_int32()
    _abi.check(_abi.lib().trstmi_optimize(int(n), int(d), ctypes.byref(p), _ptr(out), ctypes.byref(mu),
                                          ctypes.byref(best), _ptr(workspace), workspace.numel(), _stream(stream)),
               "trstmi_optimize")
    return out, mu.value, best.value


def miso_workspace_bytes(n, d, m):
    return _abi.lib().trstmi_miso_workspace_bytes(int(n), int(d), int(m))


def miso_quantize_into(codebook, n, d, channels, m, index, gain, dist, summary, workspace, stream=None):
    """trstmi_miso_quantize into caller buffers (any output may be None)."""
    _abi.check(_abi.lib().trstmi_miso_quantize(_ptr(codebook), int(n), int(d), _ptr(channels), int(m), _ptr(index),
                                               _ptr(gain), _ptr(dist), _ptr(summary), _ptr(workspace),
                                               0 if workspace is None else workspace.numel(), _stream(stream)),
               "trstmi_miso_quantize")


def miso_quantize(codebook, n, d, channels, m, per_channel=True, workspace=None, stream=None):
    """Quantise m channels (device, frame layout) with an n-word codebook
    (section III).  Returns (index int32, gain, dist) device tensors of
    length m (None unless per_channel) and a 2-element device tensor
    (mean dist, mean gain)."""
    torch = _torch()
    dev = codebook.device
    index = gain = dist = None
    if per_channel:
        index = torch.empty(max(int(m), 1), dtype=torch.int32, device=dev)
        gain = torch.empty(max(int(m), 1), dtype=torch.float64, device=dev)
        dist = torch.empty(max(int(m), 1), dtype=torch.float64, device=dev)
    summary = torch.empty(2, dtype=torch.float64, device=dev)
    if workspace is None:
        workspace = torch.empty(max(miso_workspace_bytes(n, d, m), 1), dtype=torch.uint8, device=dev)
    miso_quantize_into(codebook, n, d, channels, m, index, gain, dist, summary, workspace, stream)
    if per_channel:
        index, gain, dist = index[:m], gain[:m], dist[:m]
    return index, gain, dist, summary


def candidates(params, frame, radius, t, c0, count, explicit_z=None, out=None, stream=None):
    """The normalised FP64 candidates c0..c0+count-1 of step t (flat tensor,
    candidate i at offset i*2*d*n)."""
    torch = _torch()
    if out is None:
        out = torch.empty(count * 2 * params.d * params.n, dtype=torch.float64, device=frame.device)
    _abi.check(_abi.lib().trstmi_candidates(ctypes.byref(params), _ptr(frame), _ptr(radius), int(t), int(c0),
                                            int(count), _ptr(explicit_z), _ptr(out), _stream(stream)),
               "trstmi_candidates")
    return out


def round_bf16(x, out=None, stream=None):
    """bfloat16 bit patterns (int16 tensor) of a float64 device tensor, rounded
    as the BF16 screen rounds its inputs."""
    torch = _torch()
    x = x.contiguous()
    if out is None:
        out = torch.empty(x.numel(), dtype=torch.int16, device=x.device)
    _abi.check(_abi.lib().trstmi_round_bf16(_ptr(x), int(x.numel()), _ptr(out), _stream(stream)),
               "trstmi_round_bf16")
    return out


@dataclasses.dataclass
class DeviceState:
    frame: object
    mu: object
    radius: object
    step: object
    flags: object

    def abi(self):
        return _abi.State(self.frame.data_ptr(), self.mu.data_ptr(), self.radius.data_ptr(),
                          self.step.data_ptr(), self.flags.data_ptr())


def new_state(n, d, device="cuda"):
    torch = _torch()
    return DeviceState(
        frame=torch.zeros(2 * int(d) * int(n), dtype=torch.float64, device=device),
        mu=torch.zeros(1, dtype=torch.float64, device=device),
        radius=torch.zeros(1, dtype=torch.float64, device=device),
        step=torch.zeros(1, dtype=torch.int64, device=device),
        flags=torch.zeros(1, dtype=torch.int32, device=device),
    )


def init_haar(params, state, workspace, stream=None):
    st = state.abi()
    _abi.check(_abi.lib().trstmi_init_haar(ctypes.byref(params), ctypes.byref(st), _ptr(workspace),
                                           workspace.numel(), _stream(stream)), "trstmi_init_haar")


def step(params, state, workspace, explicit_z=None, report=None, stream=None):
    st = state.abi()
    rep = None
    if report is not None:
        rep = _abi.Report(*(0 if report.get(k) is None else report[k].data_ptr()
                            for k in ("cand_mu", "rechecked", "recheck_mu", "best")))
    _abi.check(_abi.lib().trstmi_step(ctypes.byref(params), ctypes.byref(st), _ptr(workspace), workspace.numel(),
                                      _ptr(explicit_z), ctypes.byref(rep) if rep is not None else None,
                                      _stream(stream)), "trstmi_step")


def solve(params, state, workspace, chunk=64, stream=None):
    st = state.abi()
    _abi.check(_abi.lib().trstmi_solve(ctypes.byref(params), ctypes.byref(st), _ptr(workspace), workspace.numel(),
                                       int(chunk), _stream(stream)), "trstmi_solve")


class Solver:
    """One search: parameters, device state and workspace."""

    def __init__(self, n, d, device="cuda", **kw):
        torch = _torch()
        self.params = default_params(n, d, **kw)
        self.n, self.d = int(n), int(d)
        self.state = new_state(n, d, device)
        self.workspace = torch.empty(workspace_bytes(self.params), dtype=torch.uint8, device=device)
        C = self.params.candidates
        k = max(1, self.params.recheck_topk)
        self.report = {
            "cand_mu": torch.empty(C, dtype=torch.float64, device=device),
            "rechecked": torch.empty(k, dtype=torch.int32, device=device),
            "recheck_mu": torch.empty(k, dtype=torch.float64, device=device),
            "best": torch.empty(1, dtype=torch.int32, device=device),
        }

    def init_haar(self):
        init_haar(self.params, self.state, self.workspace)
        return self

    def set_frame(self, F, mu=None, radius=None, t=0, flags=0):
        """Load a host frame (d, N) and scalars into the device state."""
        self.state.frame.copy_(frame_to_device(F, self.state.frame.device))
        if mu is not None:
            self.state.mu.fill_(float(mu))
        if radius is not None:
            self.state.radius.fill_(float(radius))
        self.state.step.fill_(int(t))
        self.state.flags.fill_(int(flags))

    def step(self, explicit_z=None, with_report=True):
        step(self.params, self.state, self.workspace, explicit_z, self.report if with_report else None)

    def solve(self, chunk=64):
        solve(self.params, self.state, self.workspace, chunk)

    def host_state(self):
        """(frame (d,N) complex128, mu, radius, step, flags) copied to the host."""
        return (frame_from_device(self.state.frame, self.n, self.d), float(self.state.mu.item()),
                float(self.state.radius.item()), int(self.state.step.item()), int(self.state.flags.item()))


def timing_enable(on=True):
    _abi.check(_abi.lib().trstmi_timing_enable(1 if on else 0), "trstmi_timing_enable")


def timing_only(kernel=None):
    """Limit timing to launches of one kernel name (None: every kernel)."""
    _abi.check(_abi.lib().trstmi_timing_only(kernel.encode() if kernel else None), "trstmi_timing_only")


def timing_reset():
    _abi.check(_abi.lib().trstmi_timing_reset(), "trstmi_timing_reset")


def timing_read(kernel):
    """(total milliseconds, timed launches) of one kernel since the last reset."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _abi.check(_abi.lib().trstmi_timing_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)),
               "trstmi_timing_read")
    return ms.value, cnt.value


class Batch:
    """Many independent searches advanced together (per step, one persistent
    launch over every candidate of every instance and one finalizing launch).  ``instances``: iterable of dicts with keys n, d and optionally seed,
    stream_id, target_mu, max_steps, waves_per_item (default: the autotuned
    table, else the library's choice)."""

    def __init__(self, instances, candidates=64, radius0=0.1, grow=2.0, shrink=0.5, radius_min=1e-12,
                 radius_max=1.0, near_tie=0.0, device="cuda"):
        torch = _torch()
        from . import autotune
        tiles = autotune.load_table()
        inst = list(instances)
        self.count = len(inst)
        self.inst = (_abi.BatchInstance * self.count)()
        for k, spec in enumerate(inst):
            I = self.inst[k]
            I.n, I.d = int(spec["n"]), int(spec["d"])
            I.seed = int(spec.get("seed", 0))
            I.stream_id = int(spec.get("stream_id", k))
            I.target_mu = float(spec.get("target_mu", 0.0))
            I.max_steps = int(spec.get("max_steps", 1000))
            w = spec.get("waves_per_item")
            I.waves_per_item = int(autotune.choose(tiles, I.n, I.d) if w is None else w)
        self.params = _abi.BatchParams(self.count, int(candidates), float(radius0), float(grow), float(shrink),
                                       float(radius_min), float(radius_max), float(near_tie))
        nbytes = _abi.lib().trstmi_batch_workspace_bytes(ctypes.byref(self.params), self.inst)
        if nbytes == 0:
            raise _abi.TrstmiError(_abi.E_INVALID_ARG, "trstmi_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.rep_mu = torch.empty(self.count * int(candidates), dtype=torch.float64, device=device)
        self.rep_best = torch.empty(self.count, dtype=torch.int32, device=device)
        self.device = device

    def _args(self):
        return ctypes.byref(self.params), self.inst, _ptr(self.workspace), self.workspace.numel()

    def init(self, stream=None):
        _abi.check(_abi.lib().trstmi_batch_init(*self._args(), _stream(stream)), "trstmi_batch_init")
        return self

    def step(self, launches=1, report=False, stream=None):
        _abi.check(_abi.lib().trstmi_batch_step(*self._args(), int(launches),
                                                _ptr(self.rep_mu) if report else None,
                                                _ptr(self.rep_best) if report else None, _stream(stream)),
                   "trstmi_batch_step")

    def run(self, chunk=16, max_chunks=1000, stream=None):
        done = ctypes.c_int32(0)
        _abi.check(_abi.lib().trstmi_batch_run(*self._args(), int(chunk), int(max_chunks), ctypes.byref(done),
                                               _stream(stream)), "trstmi_batch_run")
        return bool(done.value)

    def query(self, stream=None):
        """Host numpy arrays (mu, radius, step, flags) and the DONE count."""
        n = self.count
        mu = np.zeros(n)
        radius = np.zeros(n)
        step = np.zeros(n, dtype=np.int64)
        flags = np.zeros(n, dtype=np.int32)
        done = ctypes.c_int32(0)
        _abi.check(_abi.lib().trstmi_batch_query(*self._args(), mu.ctypes.data_as(ctypes.c_void_p),
                                                 radius.ctypes.data_as(ctypes.c_void_p),
                                                 step.ctypes.data_as(ctypes.c_void_p),
                                                 flags.ctypes.data_as(ctypes.c_void_p), ctypes.byref(done),
                                                 _stream(stream)), "trstmi_batch_query")
        return mu, radius, step, flags, done.value

    def frame(self, i, stream=None):
        """Instance i's frame as a numpy (d, N) complex128 array."""
        torch = _torch()
        n, d = self.inst[i].n, self.inst[i].d
        out = torch.empty(2 * n * d, dtype=torch.float64, device=self.device)
        _abi.check(_abi.lib().trstmi_batch_frame(*self._args(), int(i), _ptr(out), _stream(stream)),
                   "trstmi_batch_frame")
        return frame_from_device(out, n, d)
