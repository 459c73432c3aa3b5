"""Serving form: a stream of solve requests with continuous admission.

Requests (N, d, seed, arrival time) arrive over time.  A request is admitted
as soon as a slot is free and its device footprint (workspace + frame +
scalars) fits in the memory pool; it then runs on the GPU on its slot's own
HIP stream, concurrently with the requests already running, until its
coherence reaches the target (default 1.10 x the Welch bound) or its step
limit.  Frames, radii and step counters stay resident in device memory for
the whole solve; the host only polls a done flag once per chunk of
graph-captured steps.  Requests arriving while others run are admitted as
soon as slots and memory free up (no batch boundary to wait for).  A request
larger than the whole pool is rejected with a status, never queued forever.

Every result is a pure function of the request (its own seed and stream):
the same alone and in any mix.
"""

from __future__ import annotations

import bisect
import dataclasses
import math
import threading
import time
from typing import List, Optional

import numpy as np

from . import MODES, DeviceState, Solver, _torch, default_params, init_haar, solve, workspace_bytes


def welch_bound(n, d):
    """sqrt((N - d) / (d (N - 1))), 0 for N <= d."""
    return math.sqrt(max(0.0, (n - d) / (d * (n - 1))))


class OffsetAllocator:
    """First-fit allocator of 256-byte aligned ranges in [0, capacity)."""

    ALIGN = 256

    def __init__(self, capacity):
        self.capacity = int(capacity)
        self.free = [(0, self.capacity)]          # sorted (offset, size)
        self.used = 0
        self.peak = 0

    @classmethod
    def round(cls, size):
        return (int(size) + cls.ALIGN - 1) // cls.ALIGN * cls.ALIGN

    def alloc(self, size):
        size = self.round(size)
        for k, (off, sz) in enumerate(self.free):
            if sz >= size:
                if sz == size:
                    self.free.pop(k)
                else:
                    self.free[k] = (off + size, sz - size)
                self.used += size
                self.peak = max(self.peak, self.used)
                return off
        return None

    def release(self, off, size):
        size = self.round(size)
        k = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(k, (off, size))
        # merge with neighbours
        if k + 1 < len(self.free) and self.free[k][0] + self.free[k][1] == self.free[k + 1][0]:
            self.free[k] = (self.free[k][0], self.free[k][1] + self.free[k + 1][1])
            self.free.pop(k + 1)
        if k > 0 and self.free[k - 1][0] + self.free[k - 1][1] == self.free[k][0]:
            self.free[k - 1] = (self.free[k - 1][0], self.free[k - 1][1] + self.free[k][1])
            self.free.pop(k)
        self.used -= size


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
    status: str = "pending"   # pending | queued | running | done | rejected | error
    admit: float = math.nan
    finish: float = math.nan
    mu: float = math.nan
    steps: int = 0
    reached: bool = False
    error: str = ""

    @property
    def latency(self):
        return self.finish - self.arrival


def request_params(req, candidates, mode, recheck_topk, radius0, target_factor):
    target = req.target_mu if req.target_mu is not None else target_factor * welch_bound(req.n, req.d)
    return default_params(req.n, req.d, candidates=candidates, mode=mode, recheck_topk=recheck_topk,
                          seed=req.seed, stream_id=req.id & 0xFFFFFFFF, radius0=radius0, max_steps=req.max_steps,
                          target_mu=target)


def footprint(params):
    """Device bytes one request holds while admitted: workspace, frame, scalars."""
    frame = 16 * params.n * params.d
    return OffsetAllocator.round(workspace_bytes(params)) + OffsetAllocator.round(frame) + 256


class Server:
    """Continuous-admission solve server on one GPU."""

    def __init__(self, pool_bytes, max_active=8, chunk=64, candidates=64, mode="bf16", recheck_topk=8,
                 radius0=0.05, target_factor=1.10, device="cuda"):
        torch = _torch()
        self.torch = torch
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=device)
        self.alloc = OffsetAllocator(pool_bytes)
        self.max_active = int(max_active)
        # one stream per slot: a stream is never shared by two running requests
        # (each captures its chunk of steps into a graph on its own stream)
        self.free_streams = [torch.cuda.Stream(device=device) for _ in range(self.max_active)]
        self.chunk = int(chunk)
        self.candidates = int(candidates)
        self.mode = MODES.get(mode, mode)
        self.recheck_topk = int(recheck_topk)
        self.radius0 = float(radius0)
        self.target_factor = float(target_factor)
        self.lock = threading.Condition()
        self.active = 0

    def _views(self, off, params):
        """State tensors and workspace carved out of the pool at `off`."""
        torch = self.torch
        ws_bytes = OffsetAllocator.round(workspace_bytes(params))
        fr_bytes = OffsetAllocator.round(16 * params.n * params.d)
        base = self.pool[off:off + ws_bytes + fr_bytes + 256]
        ws = base[:ws_bytes]
        frame = base[ws_bytes:ws_bytes + 16 * params.n * params.d].view(torch.float64)
        sc = base[ws_bytes + fr_bytes:ws_bytes + fr_bytes + 256]
        st = DeviceState(frame=frame, mu=sc[0:8].view(torch.float64), radius=sc[8:16].view(torch.float64),
                         step=sc[16:24].view(torch.int64), flags=sc[24:28].view(torch.int32))
        return ws, st

    def _run_one(self, req, params, off, size, stream, t0):
        torch = self.torch
        try:
            ws, st = self._views(off, params)
            with torch.cuda.stream(stream):
                init_haar(params, st, ws, stream=stream)
                solve(params, st, ws, chunk=self.chunk, stream=stream)
                stream.synchronize()
                req.mu = float(st.mu.item())
                req.steps = int(st.step.item())
            req.reached = req.mu <= params.target_mu
            req.status = "done"
        except Exception as exc:  # noqa: BLE001
            req.status = "error"
            req.error = str(exc)
        req.finish = time.perf_counter() - t0
        with self.lock:
            self.alloc.release(off, size)
            self.free_streams.append(stream)
            self.active -= 1
            self.lock.notify_all()

    def run(self, requests: List[Request], poll_s=0.002, progress=None, progress_every_s=10.0):
        """Serve `requests` (arrival times relative to now).  Returns a dict of
        statistics; per-request results are written into the requests.
        `progress(text)`, if given, is called about every progress_every_s."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.id))
        t0 = time.perf_counter()
        last_report = t0
        queue = []
        threads = []
        k = 0
        while True:
            now = time.perf_counter() - t0
            if progress and time.perf_counter() - last_report >= progress_every_s:
                last_report = time.perf_counter()
                finished = sum(r.status in ("done", "rejected", "error") for r in reqs)
                progress(f"serving t={now:.1f}s finished={finished}/{len(reqs)} active={self.active} "
                         f"queued={len(queue)}")
            while k < len(reqs) and reqs[k].arrival <= now:      # arrivals
                r = reqs[k]
                k += 1
                params = request_params(r, self.candidates, self.mode, self.recheck_topk, self.radius0,
                                        self.target_factor)
                size = footprint(params)
                if size > self.alloc.capacity:
                    r.status = "rejected"
                    r.error = f"footprint {size} B exceeds the pool ({self.alloc.capacity} B)"
                    r.finish = now
                    continue
                r.status = "queued"
                queue.append((r, params, size))
            with self.lock:
                while queue and self.active < self.max_active:   # admission, first in line first
                    r, params, size = queue[0]
                    off = self.alloc.alloc(size)
                    if off is None:
                        break
                    queue.pop(0)
                    self.active += 1
                    r.status = "running"
                    r.admit = time.perf_counter() - t0
                    stream = self.free_streams.pop()
                    th = threading.Thread(target=self._run_one, args=(r, params, off, size, stream, t0),
                                          daemon=True)
                    threads.append(th)
                    th.start()
                if k == len(reqs) and not queue and self.active == 0:
                    break
                wait = poll_s
                if k < len(reqs):
                    wait = min(max(0.0, reqs[k].arrival - (time.perf_counter() - t0)), 0.05)
                if self.active:
                    self.lock.wait(timeout=max(wait, 1e-4))
            if not self.active:
                time.sleep(wait)
        for th in threads:
            th.join()
        wall = time.perf_counter() - t0
        return summarize(reqs, wall, self.candidates, self.alloc.peak, self.alloc.capacity)


def summarize(reqs, wall, candidates, peak_bytes, cap_bytes):
    done = [r for r in reqs if r.status == "done"]
    lat = np.array([r.latency for r in done]) if done else np.array([math.nan])
    evals = sum(r.steps * candidates for r in done)
    return {
        "requests": len(reqs),
        "done": len(done),
        "rejected": sum(r.status == "rejected" for r in reqs),
        "errors": sum(r.status == "error" for r in reqs),
        "reached_target": sum(r.reached for r in done),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_queue_s": float(np.mean([r.admit - r.arrival for r in done])) if done else math.nan,
        "evals_per_s": evals / wall if wall > 0 else math.nan,
        "wall_s": wall,
        "median_mu_over_welch": float(np.median([r.mu / welch_bound(r.n, r.d) for r in done])) if done else math.nan,
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
