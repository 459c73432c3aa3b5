"""Serving form: a stream of solve requests served by continuous batching.

The server itself is native (the library's trstmi_server_* entry points):
one engine thread keeps every admitted request in a device table and
advances all of them together, one launch of each step kernel per group of
requests with the same d; after each chunk of steps it reads back every
request's state at once, retires the finished ones and admits the requests
at the head of the queue whose device footprint (workspace, frame, state
scalars) fits in the caller's pool.  A request larger than the whole pool is
rejected at once.  This module submits requests at their arrival times and
collects the results.

Every result is a pure function of the request (its own seed and stream id):
the same alone, in any mix, and as a single solve gives it.
"""

from __future__ import annotations

import ctypes
import dataclasses
import math
import time
import weakref
from typing import List, Optional

import numpy as np

from . import MODES, Solver, _abi, _torch, default_params


def welch_bound(n, d):
    """sqrt((N - d) / (d (N - 1))), 0 for N <= d (the library's value)."""
    return float(_abi.lib().trstmi_welch_bound(int(n), int(d)))


@dataclasses.dataclass
class Request:
    id: int
    arrival: float            # seconds after the start of the run
    n: int
    d: int
    seed: int = 0
    target_mu: Optional[float] = None   # None: target_factor x Welch
    max_steps: int = 20000
    # results
    status: str = "pending"   # pending | queued | running | done | rejected | error | cancelled
    admit: float = math.nan
    finish: float = math.nan
    mu: float = math.nan
    steps: int = 0
    reached: bool = False
    error: str = ""

    @property
    def latency(self):
        return self.finish - self.arrival


def _destroy(handle, pool):
    _abi.lib().trstmi_server_destroy(handle)
    del pool


_STATUS = {_abi.REQ_QUEUED: "queued", _abi.REQ_RUNNING: "running", _abi.REQ_DONE: "done", _abi.REQ_ERROR: "error",
           _abi.REQ_REJECTED: "rejected", _abi.REQ_CANCELLED: "cancelled"}


def request_params(req, candidates, mode, recheck_topk, radius0, target_factor):
    """The solve parameters the server uses for a request (stream id = the
    request's id)."""
    target = req.target_mu if req.target_mu is not None else target_factor * welch_bound(req.n, req.d)
    return default_params(req.n, req.d, candidates=candidates, mode=mode, recheck_topk=recheck_topk,
                          seed=req.seed, stream_id=req.id & 0xFFFFFFFF, radius0=radius0, max_steps=req.max_steps,
                          target_mu=target)


def footprint(params):
    """Device bytes one request holds while admitted: workspace, frame, scalars."""
    return int(_abi.lib().trstmi_request_footprint(ctypes.byref(params)))


class Server:
    """Continuous-admission solve server on one GPU (the native server over a
    torch-allocated pool)."""

    def __init__(self, pool_bytes, max_active=64, chunk=64, candidates=64, mode="bf16", recheck_topk=8,
                 radius0=0.05, target_factor=1.10, device="cuda"):
        """pool_bytes: device bytes for the admitted requests (the engine's
        table for max_active rows is added on top)."""
        torch = _torch()
        table = int(_abi.lib().trstmi_server_table_bytes(int(max_active)))
        if table == 0:
            raise ValueError("max_active must be in [1, 1024]")
        pool_bytes = int(pool_bytes) + table
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=device)
        self.candidates = int(candidates)
        self.mode = MODES.get(mode, mode)
        self.target_factor = float(target_factor)
        p = _abi.ServerParams(ctypes.c_void_p(self.pool.data_ptr()), int(pool_bytes), int(max_active), int(chunk),
                              int(candidates), int(self.mode), int(recheck_topk), 0, float(radius0),
                              float(target_factor))
        handle = ctypes.c_void_p()
        _abi.check(_abi.lib().trstmi_server_create(ctypes.byref(p), ctypes.byref(handle)), "trstmi_server_create")
        self.handle = handle
        # destroy (join the engine thread) when the server is collected or at
        # interpreter exit, before the HIP runtime goes away; the pool stays
        # referenced until then
        self._finalizer = weakref.finalize(self, _destroy, handle, self.pool)

    def close(self):
        """Let running requests finish, cancel queued ones, stop the engine."""
        self._finalizer()

    def submit(self, req):
        rq = _abi.ServeRequest(int(req.n), int(req.d), int(req.seed), int(req.id) & 0xFFFFFFFF,
                               math.nan if req.target_mu is None else float(req.target_mu), int(req.max_steps))
        rid = ctypes.c_int64()
        _abi.check(_abi.lib().trstmi_server_submit(self.handle, ctypes.byref(rq), ctypes.byref(rid)),
                   "trstmi_server_submit")
        return rid.value

    def result(self, rid, wait_s=0.0):
        """(result struct, message) of a submitted request, waiting up to
        wait_s seconds (< 0: until it finishes)."""
        out = _abi.RequestResult()
        if wait_s == 0.0:
            st = _abi.lib().trstmi_server_poll(self.handle, int(rid), ctypes.byref(out))
        else:
            st = _abi.lib().trstmi_server_wait(self.handle, int(rid), float(wait_s), ctypes.byref(out))
        _abi.check(st, "trstmi_server_poll")
        msg = _abi.lib().trstmi_last_error().decode(errors="replace") if out.status in (
            _abi.REQ_ERROR, _abi.REQ_REJECTED) else ""
        return out, msg

    def stats(self):
        s = _abi.ServerStats()
        _abi.check(_abi.lib().trstmi_server_get_stats(self.handle, ctypes.byref(s)), "trstmi_server_get_stats")
        return s

    def run(self, requests: List[Request], progress=None, progress_every_s=10.0, warmup=0):
        """Serve `requests`, each submitted at its arrival time (relative to
        now).  Returns a dict of statistics (the first `warmup` arrivals are
        left out of the latency statistics); per-request results are written
        into the requests.  `progress(text)`, if given, is called about every
        progress_every_s while requests are outstanding."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.id))
        t0 = time.perf_counter()
        ids = []
        for r in reqs:
            delay = r.arrival - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            ids.append(self.submit(r))
            r.status = "queued"
        last = time.perf_counter()
        for r, rid in zip(reqs, ids):
            while True:
                out, msg = self.result(rid, wait_s=1.0)
                if out.status >= _abi.REQ_DONE:
                    break
                if progress and time.perf_counter() - last >= progress_every_s:
                    last = time.perf_counter()
                    s = self.stats()
                    progress(f"serving t={last - t0:.1f}s active={s.active} queued={s.queued}")
            _abi.lib().trstmi_server_forget(self.handle, int(rid))
            r.status = _STATUS[out.status]
            r.error = msg
            r.mu = out.mu
            r.steps = int(out.steps)
            r.reached = bool(out.reached)
            if out.status in (_abi.REQ_REJECTED, _abi.REQ_CANCELLED):
                r.finish = r.arrival
            else:
                r.admit = r.arrival + out.queue_s
                r.finish = r.admit + out.run_s
        wall = time.perf_counter() - t0
        s = self.stats()
        return summarize(reqs, wall, self.candidates, s.pool_peak, s.pool_capacity, warmup)


def _pct(values, q):
    return float(np.percentile(np.array(values), q)) if len(values) else None


def summarize(reqs, wall, candidates, peak_bytes, cap_bytes, warmup=0):
    """Latency = finish - arrival: over every finished request (time to the
    target or to the step cap) and over those that reached the target (time
    to target); queue = admission - arrival; evals = steps x candidates, and
    the screen's algorithmic flops 8 d N (N - 1) / 2 per eval.  The first
    `warmup` requests by arrival count towards throughput but not towards the
    latency, queue and target statistics.  An empty statistic is None."""
    done_all = [r for r in reqs if r.status == "done"]
    measured = set(id(r) for r in sorted(reqs, key=lambda r: (r.arrival, r.id))[warmup:])
    done = [r for r in done_all if id(r) in measured]
    reached = [r for r in done if r.reached]
    evals = sum(r.steps * candidates for r in done_all)
    flops = sum(r.steps * candidates * 4.0 * r.d * r.n * (r.n - 1) for r in done_all)
    queue = [r.admit - r.arrival for r in done]
    by_d = {}
    for r in done:
        e = by_d.setdefault(str(r.d), {"done": 0, "reached_target": 0})
        e["done"] += 1
        e["reached_target"] += int(r.reached)
    return {
        "requests": len(reqs),
        "warmup_requests": int(warmup),
        "done": len(done_all),
        "rejected": sum(r.status == "rejected" for r in reqs),
        "errors": sum(r.status == "error" for r in reqs),
        "measured": len(done),
        "reached_target": len(reached),
        "reached_by_d": by_d,
        "p50_latency_s": _pct([r.latency for r in done], 50),
        "p99_latency_s": _pct([r.latency for r in done], 99),
        "p50_time_to_target_s": _pct([r.latency for r in reached], 50),
        "p99_time_to_target_s": _pct([r.latency for r in reached], 99),
        "mean_queue_s": float(np.mean(queue)) if done else None,
        "p50_queue_s": _pct(queue, 50),
        "p99_queue_s": _pct(queue, 99),
        "evals_per_s": evals / wall if wall > 0 else None,
        "screen_tflops": flops / wall / 1e12 if wall > 0 else None,
        "wall_s": wall,
        "median_mu_over_welch": float(np.median([r.mu / welch_bound(r.n, r.d) for r in done])) if done else None,
        "pool_peak_bytes": int(peak_bytes),
        "pool_cap_bytes": int(cap_bytes),
        "first_error": next((r.error for r in reqs if r.status == "error"), ""),
    }


def solve_alone(req, candidates=64, mode="bf16", recheck_topk=8, radius0=0.05, target_factor=1.10, chunk=64):
    """The same request solved by itself (reference for the mix test).
    Returns (frame, mu, radius, step, flags)."""
    params = request_params(req, candidates, MODES.get(mode, mode), recheck_topk, radius0, target_factor)
    s = Solver(req.n, req.d, candidates=candidates, mode=params.mode, recheck_topk=recheck_topk, seed=params.seed,
               stream_id=params.stream_id, radius0=radius0, max_steps=params.max_steps, target_mu=params.target_mu)
    s.init_haar()
    s.solve(chunk)
    return s.host_state()
