#!/usr/bin/env python
"""Throughput of the candidate-coherence step on one MI355X.

A step is one pass of the whole path over one batch of synthetic input:
C = 128 trust-region perturbations of a Haar-random frame of N = 4096 unit
vectors in C^64, renormalised, screened from BF16 inputs on MFMA (FP32
accumulation), the 8 best re-evaluated exactly in FP64 (certified tile
pruning), select / accept / radius update, commit.  The frame is resident in
HBM when the timed region starts.

Output: one JSON line.  ``value`` is candidate evaluations per second over
the timed steps; ``roofline`` is the BF16 Gram kernel's algorithmic
TFLOP/s (8 d N(N-1)/2 flops per candidate) over its average launch time,
measured with HIP events on its stream inside the timed region;
``cpu_baseline`` is the numpy FP64 oracle on a bounded sample of the same
workload on this host.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"bf16": 2516.6, "fp32": 157.3, "fp64": 78.6}   # MI355X dense MFMA
GRAM_KERNEL = {"bf16": "gram_bf16", "fp32": "gram_f32", "fp64": "gram_f64"}
KERNEL_SOURCE = {"gram_bf16": "gram_bf16.hip", "gram_f32": "gram_f32.hip", "gram_f64": "gram_f64.hip"}
METRIC = "candidate coherence evals/s at N=4096,d=64 (% roofline); p50/p99 solve latency"


def log(text):
    print(f"[bench] {text}", file=sys.stderr, flush=True)


def flops_per_eval(n, d):
    """Algorithmic flops of one candidate's Gram + coherence: the strict upper
    triangle has n(n-1)/2 complex inner products of length d, 8 real flops per
    complex multiply-add."""
    return 8 * d * n * (n - 1) // 2


def kernel_sha(name):
    path = os.path.join(ROOT, "paper_2207_06374_amd", "csrc", KERNEL_SOURCE[name])
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(name):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; otherwise None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get(name)
    if not rec or rec.get("source_sha") != kernel_sha(name):
        return None
    return rec.get("bytes_per_launch")


STEP_KERNELS = ("perturb", "gram_f64", "gram_f32", "gram_bf16", "topk", "perturb_recheck", "recheck", "select",
                "commit")


def warm_up(lib, torch, s, mode, min_steps, min_s=1.0, max_s=20.0, window=200):
    """Untimed steps until the Gram kernel's average launch time is steady:
    at least ``min_steps`` steps and ``min_s`` seconds, then windows of
    ``window`` steps until two consecutive window averages agree within 1 %
    (at most ``max_s`` seconds).  Clocks ramp up over the first second of a
    fresh process; timing before that reads them low."""
    t0 = time.perf_counter()
    for _ in range(min_steps):
        s.step(with_report=False)
    torch.cuda.synchronize()
    prev = None
    lib.timing_only(GRAM_KERNEL[mode])
    while True:
        lib.timing_reset()
        lib.timing_enable(True)
        for k in range(window):
            s.step(with_report=False)
            if k % 32 == 31:
                torch.cuda.synchronize()
        torch.cuda.synchronize()
        lib.timing_enable(False)
        ms, cnt = lib.timing_read(GRAM_KERNEL[mode])
        avg = ms / max(cnt, 1)
        el = time.perf_counter() - t0
        if el >= max_s or (el >= min_s and prev is not None and abs(avg - prev) <= 0.01 * prev):
            break
        prev = avg
    lib.timing_only(None)
    lib.timing_reset()
    return {"seconds": time.perf_counter() - t0, "last_window_gram_us": 1e3 * avg}


def run_mode(lib, torch, wl, mode, steps, warmup, topk=8, breakdown_steps=10, min_warm_s=1.0, window=200):
    """Timed steps with HIP events around the Gram kernel only (the other
    kernels' events would add to the step), after a warm-up that runs until
    the Gram time is steady; then a few steps with every kernel timed for the
    per-kernel breakdown."""
    s = lib.Solver(wl.n, wl.d, candidates=wl.candidates, mode=mode, recheck_topk=topk, radius0=wl.radius0,
                   max_steps=2 ** 32 - 1, seed=wl.seed, stream_id=wl.stream_id)
    s.init_haar()
    warm = warm_up(lib, torch, s, mode, warmup, min_s=min_warm_s, window=window)
    torch.cuda.synchronize()
    lib.timing_reset()
    lib.timing_only(GRAM_KERNEL[mode])
    lib.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        s.step(with_report=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.timing_enable(False)
    ms, cnt = lib.timing_read(GRAM_KERNEL[mode])
    g = {"avg_us": 1e3 * ms / cnt, "launches": cnt}
    mu = float(s.state.mu.item())
    lib.timing_reset()
    lib.timing_only(None)
    lib.timing_enable(True)
    for _ in range(breakdown_steps):
        s.step(with_report=False)
    torch.cuda.synchronize()
    lib.timing_enable(False)
    kernels = {}
    for name in STEP_KERNELS:
        kms, kcnt = lib.timing_read(name)
        if kcnt:
            kernels[name] = {"avg_us": 1e3 * kms / kcnt, "launches": kcnt}
    elapsed = t1 - t0
    evals = wl.candidates * steps / elapsed
    flops_launch = wl.candidates * flops_per_eval(wl.n, wl.d)
    achieved = flops_launch / (g["avg_us"] * 1e-6) / 1e12
    del s
    torch.cuda.empty_cache()
    return {
        "evals_per_s": evals,
        "ms_per_step": 1e3 * elapsed / steps,
        "final_mu": mu,
        "gram": g,
        "kernels": kernels,
        "gram_tflops": achieved,
        "gram_frac": achieved / PEAK_TFLOPS[mode],
        "flops_per_launch": flops_launch,
        "warmup": warm,
    }


def run_small_solve(lib, torch, wl, chunk=64):
    """The small workload as one full solve: N=16 in C^4, 64 candidates,
    radius 0.1, 2000 FP64 steps from the Haar start (seed 0), graph-captured
    chunks; wall time of trstmi_solve and the final coherence."""
    s = lib.Solver(wl.n, wl.d, candidates=wl.candidates, mode="fp64", radius0=wl.radius0, max_steps=wl.steps,
                   seed=wl.seed, stream_id=wl.stream_id)
    s.init_haar()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.solve(chunk)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    F, mu, radius, t, flags = s.host_state()
    return {"workload": f"N={wl.n}, d={wl.d}, {wl.candidates} candidates, radius {wl.radius0}, {wl.steps} FP64 steps, "
                        f"Haar start seed {wl.seed}; trstmi_solve with graph-captured chunks of {chunk} steps",
            "gpu_wall_s": wall, "steps": t, "final_mu": mu, "final_radius": radius,
            "welch": math.sqrt((wl.n - wl.d) / (wl.d * (wl.n - 1)))}


def run_equal_mu(lib, torch, wl, probe_steps=300, cap_factor=4, chunk=16):
    """Seconds for the FP64, FP32 and BF16-screen forms to reach one common
    coherence from the same Haar start (seed 0) at N=4096, d=64, C=128.  The
    target T is the exact coherence the BF16 form reaches after
    ``probe_steps`` steps; each form then solves from the start with target
    T (the FP32 form with T - 4e-6, so that its FP32 coherence, within 2e-6
    of the exact one, certifies mu <= T).  Every final frame is re-evaluated
    with the library's FP64 coherence; the frames are returned for the
    oracle's check in the CPU leg."""
    probe = lib.Solver(wl.n, wl.d, candidates=wl.candidates, mode="bf16", radius0=wl.radius0,
                       max_steps=probe_steps, seed=wl.seed, stream_id=wl.stream_id)
    probe.init_haar()
    probe.solve(chunk)
    target = float(probe.state.mu.item())
    del probe
    out, frames = {"target_mu": target, "probe_steps": probe_steps}, {}
    for mode in ("bf16", "fp32", "fp64"):
        goal = target - 4e-6 if mode == "fp32" else target
        s = lib.Solver(wl.n, wl.d, candidates=wl.candidates, mode=mode, radius0=wl.radius0,
                       max_steps=cap_factor * probe_steps, seed=wl.seed, stream_id=wl.stream_id, target_mu=goal)
        s.init_haar()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.solve(chunk)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        F, mu, radius, t, flags = s.host_state()
        mu64 = float(lib.coherence(s.state.frame, wl.n, wl.d, lib.MODE_FP64).item())
        out[mode] = {"seconds": wall, "steps": t, "state_mu": mu, "fp64_mu": mu64, "reached": mu64 <= target,
                     "evals_per_s": wl.candidates * t / wall}
        frames[mode] = F
        log(f"equal mu {mode}: {t} steps in {wall:.2f} s, FP64 mu {mu64:.10f} (target {target:.10f})")
        del s
        torch.cuda.empty_cache()
    return out, frames


def run_batched(lib, torch, steps, warmup, count=512, candidates=64, late_at=1000, clock_warmup_s=0.5):
    """The batched workload: 512 independent searches, d uniform in {3..16},
    N uniform in [d+1, d^2], 64 candidates each, one persistent launch (plus a
    finalizing launch) per step; candidate evaluations per second over all
    instances.  The cost of a step grows as the searches converge (more pairs
    crowd within the screen's bound of each maximum and go to the FP64
    recheck), so two figures: the first `steps` steps from the Haar starts,
    and `steps` steps from step `late_at` on, when most instances sit at the
    smallest radius (late_at <= 0: no second figure).  The clock is warmed
    up on a separate batch first, for clock_warmup_s seconds."""
    import inputs
    specs = [{"n": n, "d": d, "seed": 0, "stream_id": k, "max_steps": 10 ** 9}
             for k, (d, n) in enumerate(inputs.batched_instances(count, seed=0))]
    if clock_warmup_s > 0:
        w = lib.Batch(specs, candidates=candidates, radius0=0.1).init()
        t_w = time.perf_counter()
        while time.perf_counter() - t_w < clock_warmup_s:
            w.step(20)
            torch.cuda.synchronize()
        del w
    flops = sum(candidates * flops_per_eval(n, d) for d, n in inputs.batched_instances(count, seed=0))

    def timed(b):
        lib.timing_reset()
        lib.timing_enable(True)
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lib.timing_enable(False)
        ms, cnt = lib.timing_read("batch_step")
        avg_us = 1e3 * ms / cnt
        return {
            "evals_per_s": count * candidates * steps / (t1 - t0),
            "ms_per_step": 1e3 * (t1 - t0) / steps,
            "kernel_avg_us": avg_us,
            "algorithmic_tflops": flops / (avg_us * 1e-6) / 1e12,
            # against the FP32 peak (the precision the screen stands for) and
            # against what the split arithmetic allows (a third of the BF16 peak)
            "frac_fp32_peak": flops / (avg_us * 1e-6) / 1e12 / PEAK_TFLOPS["fp32"],
            "frac_split_bf16_peak": flops / (avg_us * 1e-6) / 1e12 / (PEAK_TFLOPS["bf16"] / 3),
        }

    b = lib.Batch(specs, candidates=candidates, radius0=0.1).init()
    b.step(warmup)
    torch.cuda.synchronize()
    out = timed(b)
    out["steps_timed"] = f"{warmup + 1}..{warmup + steps} from the Haar starts"
    done = warmup + steps
    if late_at > 0:
        if late_at > done:
            b.step(late_at - done)
            torch.cuda.synchronize()
        late = timed(b)
        late["steps_timed"] = f"{max(late_at, done) + 1}..{max(late_at, done) + steps}"
        late["mean_mu"] = float(b.query()[0].mean())
        out["late"] = late
    out["workload"] = (f"{count} instances, d in {{3..16}}, N in [d+1, d^2], {candidates} candidates each, "
                       "FP32-class screen on BF16 MFMA (each FP32 value as hi + lo bfloat16 parts, three products) + "
                       "certified FP64 pair recheck, one persistent launch and one finalizing launch per step")
    return out


def run_smooth_max(lib, torch, wl, evals, delta=1e-3):
    """The smooth maximum of section IV on the throughput shape (one Haar
    frame, N=4096, d=64): FP64 normalisation, one FP64 MFMA pass over the
    upper-triangle tiles (block maxima and rescaled sums) and the fixed-order
    finish; then the value with its gradient with respect to the frame."""
    import numpy as np
    s = lib.Solver(wl.n, wl.d, candidates=8, mode="fp64", seed=wl.seed, stream_id=wl.stream_id)
    s.init_haar()
    frame = s.state.frame
    out = torch.empty(2, dtype=torch.float64, device=frame.device)
    ws = torch.empty(lib.lse_workspace_bytes(wl.n, wl.d), dtype=torch.uint8, device=frame.device)
    for _ in range(3):
        lib.lse(frame, wl.n, wl.d, delta, True, out, ws)
    torch.cuda.synchronize()
    lib.timing_reset()
    lib.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(evals):
        lib.lse(frame, wl.n, wl.d, delta, True, out, ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.timing_enable(False)
    us = {}
    for k in ("lse_pass",):
        ms, cnt = lib.timing_read(k)
        us[k] = 1e3 * ms / cnt
    flops = flops_per_eval(wl.n, wl.d)  # the one pass over the upper-triangle tiles
    s_val, f_val = out.cpu().numpy().tolist()
    # value and gradient with respect to the frame (the paper's optimiser's step)
    grad = torch.empty_like(frame)
    gws = torch.empty(lib.lse_grad_workspace_bytes(wl.n, wl.d), dtype=torch.uint8, device=frame.device)
    for _ in range(2):
        lib.lse_grad(frame, wl.n, wl.d, delta, out, grad, gws)
    torch.cuda.synchronize()
    lib.timing_reset()
    lib.timing_enable(True)
    t2 = time.perf_counter()
    for _ in range(evals):
        lib.lse_grad(frame, wl.n, wl.d, delta, out, grad, gws)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    lib.timing_enable(False)
    ms, cnt = lib.timing_read("lse_grad")
    grad_us = 1e3 * ms / cnt
    # exact Hessian-vector product along a seeded direction (one more tile
    # pass on FP64 MFMA after the value)
    V = lib.frame_to_device(np.random.default_rng(1).standard_normal((wl.d, wl.n))
                            + 1j * np.random.default_rng(2).standard_normal((wl.d, wl.n)))
    hv = torch.empty_like(frame)
    hws = torch.empty(lib.lse_hvp_workspace_bytes(wl.n, wl.d), dtype=torch.uint8, device=frame.device)
    for _ in range(2):
        lib.lse_hvp(frame, V, wl.n, wl.d, delta, out, hv, hws)
    torch.cuda.synchronize()
    lib.timing_reset()
    lib.timing_enable(True)
    t6 = time.perf_counter()
    for _ in range(evals):
        lib.lse_hvp(frame, V, wl.n, wl.d, delta, out, hv, hws)
    torch.cuda.synchronize()
    t7 = time.perf_counter()
    lib.timing_enable(False)
    ms, cnt = lib.timing_read("lse_hv")
    hv_us = 1e3 * ms / cnt
    hv_flop = 48 * wl.d * wl.n * (wl.n - 1)  # per ordered pair: six real products of length 2d forward, six back
    # trust-region steps (Steihaug CG with exact Hessian products) from the
    # same frame; each CG iteration costs one Hessian-vector product
    Y = frame.clone()
    tws = torch.empty(lib.tr_workspace_bytes(wl.n, wl.d), dtype=torch.uint8, device=frame.device)
    radius, tr_reps = 0.05, []
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    for _ in range(3):
        rep = lib.tr_step(Y, wl.n, wl.d, delta, radius, cg_max_iter=5, workspace=tws)
        tr_reps.append(rep)
        radius = rep["new_radius"]
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    grad_calls = sum(1 + 2 * r["cg_iters"] for r in tr_reps)
    n, d = wl.n, wl.d
    grad_alg = 8 * d * n * (n - 1) // 2 + 8 * d * n * (n - 1)   # Gram once + D = Phi (W o G)
    grad_issued = 16 * d * n * n                                  # the kernel forms G over the full square
    return {
        "workload": f"F_(s,delta) of |G|^2 over j<k, N={wl.n}, d={wl.d}, delta={delta}, FP64 (Haar frame seed 0)",
        "ms_per_eval": 1e3 * (t1 - t0) / evals,
        "evals_per_s": evals / (t1 - t0),
        "pass_us": us["lse_pass"],
        "pass_frac_fp64_peak": flops / (us["lse_pass"] * 1e-6) / 1e12 / PEAK_TFLOPS["fp64"],
        "s": s_val,
        "F": f_val,
        "grad_ms_per_eval": 1e3 * (t3 - t2) / evals,
        "grad_pass_us": grad_us,
        "grad_algorithmic_flop": grad_alg,
        "grad_issued_flop": grad_issued,
        "grad_pass_frac_fp64_peak": grad_alg / (grad_us * 1e-6) / 1e12 / PEAK_TFLOPS["fp64"],
        "grad_pass_issued_frac_fp64_peak": grad_issued / (grad_us * 1e-6) / 1e12 / PEAK_TFLOPS["fp64"],
        "hvp_ms_per_call": 1e3 * (t7 - t6) / evals,
        "hv_pass_us": hv_us,
        "hv_flop": hv_flop,
        "hv_pass_frac_fp64_peak": hv_flop / (hv_us * 1e-6) / 1e12 / PEAK_TFLOPS["fp64"],
        "tr_steps": len(tr_reps),
        "tr_ms_per_step": 1e3 * (t5 - t4) / len(tr_reps),
        "tr_ms_per_gradient_call": 1e3 * (t5 - t4) / grad_calls,
        "tr_cg_iters": [r["cg_iters"] for r in tr_reps],
        "tr_cg_exit": [r["cg_exit"] for r in tr_reps],
        "tr_F": [tr_reps[0]["f_old"]] + [r["f_new"] if r["accepted"] else r["f_old"] for r in tr_reps],
    }


def run_miso(lib, torch, n, d, m, evals):
    """The beamforming-codebook evaluation of section III: m CN(0, I_d)
    channels quantised with an n-word codebook (normalise the codebook, FP64
    MFMA products with a fused argmax, fixed-order means of the squared
    chordal distance and the gain)."""
    import inputs
    C = lib.frame_to_device(inputs.random_frame(n, d, seed=1, scale_spread=False))
    H = lib.frame_to_device(inputs.miso_channels(m, d, seed=2))
    index = torch.empty(m, dtype=torch.int32, device=C.device)
    gain = torch.empty(m, dtype=torch.float64, device=C.device)
    dist = torch.empty(m, dtype=torch.float64, device=C.device)
    summary = torch.empty(2, dtype=torch.float64, device=C.device)
    ws = torch.empty(lib.miso_workspace_bytes(n, d, m), dtype=torch.uint8, device=C.device)

    def call():
        lib.miso_quantize_into(C, n, d, H, m, index, gain, dist, summary, ws)

    for _ in range(2):
        call()
    torch.cuda.synchronize()
    lib.timing_reset()
    lib.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(evals):
        call()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.timing_enable(False)
    ms, cnt = lib.timing_read("miso")
    us = 1e3 * ms / cnt
    flops = 8 * d * n * m                    # Re and Im of every <phi_i, h_j>: 2 x 2d multiply-adds
    D, g = summary.cpu().numpy().tolist()
    return {"workload": f"{m} CN(0, I_{d}) channels, codebook of {n} unit vectors in C^{d}, FP64",
            "ms_per_eval": 1e3 * (t1 - t0) / evals, "channels_per_s": m * evals / (t1 - t0),
            "kernel_us": us, "tflops": flops / (us * 1e-6) / 1e12,
            "frac_fp64_peak": flops / (us * 1e-6) / 1e12 / PEAK_TFLOPS["fp64"],
            "distortion": D, "mean_gain": g}


def run_table2(lib, dims):
    """The paper's optimiser (Alg. 2: delta continuation, L = 2 d^2 random
    restarts, trust-region steps) at N = d^2: the coherence reached and the
    wall time, beside the values Table II prints (upper bounds, rounded up
    at the fourth decimal)."""
    import os
    printed = {}
    for line in open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                                  "table2_trstmi_mu.txt")):
        if line.strip() and not line.startswith("#"):
            d, n, mu = line.split()
            printed[int(d)] = float(mu)
    rows = []
    for d in dims:
        n = d * d
        t0 = time.perf_counter()
        _, mu, best = lib.optimize(n, d)
        rows.append({"d": d, "n": n, "restarts": 2 * d * d, "mu": mu, "printed_mu": printed.get(d),
                     "welch": math.sqrt((n - d) / (d * (n - 1))), "seconds": time.perf_counter() - t0})
        log(f"table II d={d}: mu={mu:.10f} in {rows[-1]['seconds']:.1f} s")
    return rows


def run_serving(lib, count, max_steps, pool_gib, slots, target_factor=1.10, warmup=0, chunk=32):
    """The serving workload: Poisson arrivals (mean gap 5 ms), d in
    {8, 16, 32, 64, 128}, N uniform in [2d, 8d], each solved to
    target_factor x Welch or max_steps with BF16-screened / FP64-verified
    steps, admitted by device footprint into a capped pool and advanced by the
    continuous-batching engine."""
    import inputs
    from paper_2207_06374_amd import serve
    reqs = [serve.Request(id=r["id"], arrival=r["arrival"], n=r["n"], d=r["d"], seed=r["seed"], max_steps=max_steps)
            for r in inputs.serving_requests(count, seed=1)]
    srv = serve.Server(pool_bytes=int(pool_gib * 2 ** 30), max_active=slots, chunk=chunk, candidates=64, mode="bf16",
                       target_factor=target_factor)
    stats = srv.run(reqs, progress=log, warmup=warmup)
    srv.close()
    stats["target_factor"] = target_factor
    stats["workload"] = (f"{count} requests ({warmup} warm-up), Poisson arrivals mean gap 5 ms (200 req/s), d in {{8,16,32,64,128}}, "
                         f"N in [2d, 8d], target {target_factor} x Welch or {max_steps} steps, 64 candidates, BF16 screen + "
                         f"top-8 FP64 recheck, pool {pool_gib} GiB, engine with {slots} rows and {chunk}-step chunks")
    return stats


def serving_in_child(args, target_factor):
    """The serving leg in a child process of its own (the same script with
    --serving-child): the engine's native thread and its device state live
    and end there, and a failure of that process is reported in the result
    instead of ending the benchmark."""
    import subprocess
    cmd = [sys.executable, "-u", os.path.abspath(__file__), "--serving-child",
           "--serving-requests", str(args.serving_requests), "--serving-max-steps", str(args.serving_max_steps),
           "--serving-pool-gib", str(args.serving_pool_gib), "--serving-slots", str(args.serving_slots),
           "--serving-target-factor", repr(target_factor), "--serving-warmup", str(args.serving_warmup)]
    try:
        r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=1800)
    except subprocess.TimeoutExpired:
        return {"requests": args.serving_requests, "error": "the serving leg's process did not finish in 1800 s"}
    lines = [x for x in r.stdout.splitlines() if x.startswith("{")]
    if r.returncode != 0 or not lines:
        return {"requests": args.serving_requests,
                "error": f"the serving leg's process exited with status {r.returncode}"}
    return json.loads(lines[-1])


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _blas_info():
    from threadpoolctl import threadpool_info
    for i in threadpool_info():
        if i.get("user_api") == "blas":
            return {"library": i.get("internal_api"), "version": i.get("version"), "threads": i.get("num_threads"),
                    "architecture": i.get("architecture")}
    return {"library": "unknown", "threads": 1}


def cpu_baseline(large, medium, small, budget_s, equal_frames=None):
    """The FP64 oracle (numpy, the oracle as it stands) on bounded samples of
    the workloads, on this host's cores:

    * the throughput workload (N=4096, d=64, radius 0.05, Haar start seed 0):
      one FP64-form step with c of the 128 candidates (perturb, renormalise,
      one FP64 Gram + max per candidate, select), with every BLAS thread and
      with one;
    * the plain workload (N=1024, d=32): one FP64 step with all 256 candidates;
    * the small workload (N=16, d=4, 64 candidates): the full 2000-step solve;
    * the oracle's coherence of the final frames of the equal-coherence runs.
    """
    import numpy as np
    import oracle
    from threadpoolctl import threadpool_limits

    blas = _blas_info()
    res = {"cpu_model": _cpu_model(), "blas": blas, "host_cpus": len(os.sched_getaffinity(0))}

    def step_rate(wl, c, mode="fp64"):
        p = oracle.Params(n=wl.n, d=wl.d, candidates=c, mode=mode, radius0=wl.radius0, seed=wl.seed,
                          stream_id=wl.stream_id, max_steps=10 ** 9)
        st = oracle.haar_init(p)
        t0 = time.perf_counter()
        oracle.step(p, st)
        el = time.perf_counter() - t0
        return c / el, el

    # size the headline sample from one candidate
    _, one = step_rate(large, 1)
    c_all = int(max(2, min(large.candidates, 0.3 * budget_s / max(one, 1e-3))))
    rate_all, el_all = step_rate(large, c_all)
    with threadpool_limits(limits=1, user_api="blas"):
        _, one1 = step_rate(large, 1)
        c_one = int(max(2, min(large.candidates, 0.2 * budget_s / max(one1, 1e-3))))
        rate_one, el_one = step_rate(large, c_one)
    res.update({
        "value": rate_all,
        "unit": "evals/s",
        "cores": int(blas.get("threads") or 1),
        "kind": "oracle",
        "sample": f"one FP64-form step with {c_all} of the {large.candidates} candidates at N={large.n}, d={large.d} "
                  f"(perturb, renormalise, one FP64 Gram + max per candidate, select), numpy + "
                  f"{blas.get('library')} with {blas.get('threads')} threads; {el_all:.1f} s",
        "one_thread": {"value": rate_one, "unit": "evals/s", "candidates": c_one, "seconds": el_one},
    })
    rate_med, el_med = step_rate(medium, medium.candidates)
    res["plain_workload"] = {"value": rate_med, "unit": "evals/s", "seconds": el_med,
                             "sample": f"one FP64 step with all {medium.candidates} candidates at N={medium.n}, "
                                       f"d={medium.d}"}
    p0 = oracle.Params(n=small.n, d=small.d, candidates=small.candidates, mode="fp64", radius0=small.radius0,
                       seed=small.seed, stream_id=small.stream_id, max_steps=small.steps)
    t0 = time.perf_counter()
    st0, _ = oracle.solve(p0)
    res["small_solve"] = {"wall_s": time.perf_counter() - t0, "final_mu": st0.mu, "steps": st0.t,
                          "sample": f"the full {small.steps}-step FP64 solve at N={small.n}, d={small.d}, "
                                    f"{small.candidates} candidates"}
    if equal_frames:
        res["equal_mu_oracle_check"] = {m: oracle.coherence(np.asarray(F)) for m, F in equal_frames.items()}
    return res


def copy_calibration(torch, mib):
    """Three device-to-device copies of ``mib`` MiB: the counter readings of a
    kernel whose HBM traffic is known (read mib, write mib), which scale the
    FETCH_SIZE / WRITE_SIZE readings of the Gram kernel to bytes."""
    n = mib * 2 ** 20 // 4
    x = torch.ones(n, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--other-modes", default="fp64,fp32",
                    help="also time these plain forms on the same workload (comma list, '' for none)")
    ap.add_argument("--other-steps", type=int, default=10)
    ap.add_argument("--min-warmup-s", type=float, default=1.0,
                    help="warm up at least this long, and until the Gram time is steady, before the timed steps")
    ap.add_argument("--plain-modes", default="fp64,fp32",
                    help="forms timed on the plain workload N=1024, d=32, 256 candidates ('' for none)")
    ap.add_argument("--no-small-solve", dest="small_solve", action="store_false",
                    help="skip the full 2000-step solve of the small workload")
    ap.add_argument("--equal-mu-steps", type=int, default=300,
                    help="steps of the BF16 form that fix the common target of the equal-coherence comparison "
                         "(0: skip)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=200, help="steps of the batched workload (0: skip)")
    ap.add_argument("--batched-late-at", type=int, default=1000,
                    help="also time the batched steps from this step on, when most searches have converged (0: skip)")
    ap.add_argument("--batched-clock-warmup-s", type=float, default=0.5,
                    help="seconds of batched steps on a separate batch before the timed ones (clock warm-up)")
    ap.add_argument("--miso-evals", type=int, default=10,
                    help="codebook quantiser calls to time (4096 codewords, d = 64, 65536 channels; 0: skip)")
    ap.add_argument("--table2-dims", default="2,3,4,5",
                    help="dimensions d for the optimiser at N = d^2 (Table II comparison; empty: skip)")
    ap.add_argument("--smooth-max-evals", type=int, default=10,
                    help="evaluations of the section IV smooth maximum at the throughput shape (0: skip)")
    ap.add_argument("--serving-requests", type=int, default=96, help="requests of the serving run (0: skip)")
    ap.add_argument("--serving-max-steps", type=int, default=20000)
    ap.add_argument("--serving-pool-gib", type=float, default=1.0)
    ap.add_argument("--serving-slots", type=int, default=64)
    ap.add_argument("--serving-target-factor", type=float, default=1.10,
                    help="each request stops at this multiple of its Welch bound (or the step cap)")
    ap.add_argument("--serving-warmup", type=int, default=0,
                    help="the first arrivals left out of the serving latency statistics (throughput counts them)")
    ap.add_argument("--serving-reachable-factor", type=float, default=2.6,
                    help="a second serving run with this looser target, which part of the stream reaches within "
                         "the cap, so that time-to-target percentiles are measured (0: skip)")
    ap.add_argument("--serving-child", action="store_true",
                    help="only run the serving leg and print its statistics as one JSON line (the bench runs the "
                         "serving leg this way in a child process of its own)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run three plain device copies of MIB MiB (calibrates the HBM byte counters) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the candidate search is measured on one MI355X; "
              "multi-GPU sharding (candidates or Gram tiles across GPUs) is a design note, not a run.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        copy_calibration(torch, args.copy_calibration)
        return

    import inputs
    import paper_2207_06374_amd as lib

    if args.serving_child:
        stats = run_serving(lib, args.serving_requests, args.serving_max_steps, args.serving_pool_gib,
                            args.serving_slots, args.serving_target_factor, args.serving_warmup)
        print(json.dumps(stats), flush=True)
        return

    wl = inputs.LARGE
    main_res = run_mode(lib, torch, wl, "bf16", args.steps, args.warmup, min_warm_s=args.min_warmup_s)
    log(f"bf16 screen: {main_res['evals_per_s']:.0f} evals/s, Gram {main_res['gram']['avg_us']:.1f} us "
        f"(warm-up {main_res['warmup']['seconds']:.1f} s)")
    others = {}
    for m in [x for x in args.other_modes.split(",") if x]:
        r = run_mode(lib, torch, wl, m, args.other_steps, 2, min_warm_s=0.5, window=20)
        log(f"{m}: {r['evals_per_s']:.0f} evals/s")
        others[m] = {k: r[k] for k in ("evals_per_s", "ms_per_step", "gram_tflops", "gram_frac", "final_mu")}
        others[m]["gram_avg_us"] = r["gram"]["avg_us"]
    plain = {}
    for m in [x for x in args.plain_modes.split(",") if x]:
        r = run_mode(lib, torch, inputs.MEDIUM, m, args.other_steps, 2, min_warm_s=0.5, window=20)
        log(f"plain workload {m}: {r['evals_per_s']:.0f} evals/s, Gram {100 * r['gram_frac']:.1f} % of peak")
        plain[m] = {k: r[k] for k in ("evals_per_s", "ms_per_step", "gram_tflops", "gram_frac", "final_mu")}
        plain[m]["gram_avg_us"] = r["gram"]["avg_us"]
        plain[m]["workload"] = (f"N={inputs.MEDIUM.n}, d={inputs.MEDIUM.d}, {inputs.MEDIUM.candidates} candidates, "
                                f"radius {inputs.MEDIUM.radius0}, Haar start seed 0, {m.upper()} Gram on MFMA")
    small = run_small_solve(lib, torch, inputs.SMALL) if args.small_solve else None
    if small:
        log(f"small solve: {small['steps']} steps in {small['gpu_wall_s']:.2f} s, mu {small['final_mu']:.10f}")
    equal, equal_frames = (run_equal_mu(lib, torch, wl, args.equal_mu_steps) if args.equal_mu_steps > 0
                           else (None, None))

    smooth = run_smooth_max(lib, torch, wl, args.smooth_max_evals) if args.smooth_max_evals > 0 else None
    miso = run_miso(lib, torch, 4096, 64, 65536, args.miso_evals) if args.miso_evals > 0 else None
    table2 = run_table2(lib, [int(x) for x in args.table2_dims.split(",") if x]) if args.table2_dims else None
    batched = (run_batched(lib, torch, args.batched_steps, 2, late_at=args.batched_late_at,
                           clock_warmup_s=args.batched_clock_warmup_s) if args.batched_steps > 0 else None)
    log("batched done")
    serving = serving_in_child(args, args.serving_target_factor) if args.serving_requests > 0 else None
    serving_reachable = (serving_in_child(args, args.serving_reachable_factor)
                         if args.serving_requests > 0 and args.serving_reachable_factor > 0 else None)

    g = main_res["gram"]
    traffic = load_traffic("gram_bf16")
    line = {
        "metric": METRIC,
        "value": main_res["evals_per_s"],
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": "N=4096 unit vectors in C^64, 128 candidates/step, radius 0.05, Haar start seed 0; "
                        "BF16-input MFMA screen, top-8 FP64 recheck (certified tile pruning), FP64 accept",
            "n": wl.n, "d": wl.d, "candidates": wl.candidates, "recheck_topk": 8, "radius0": wl.radius0,
            "recheck_dtype": "f64",
        },
        "roofline": {
            "bound": "mfma",
            "kernel": "gram_bf16",
            "achieved": main_res["gram_tflops"],
            "peak": PEAK_TFLOPS["bf16"],
            "unit": "TFLOP/s",
            "frac": main_res["gram_frac"],
            "traffic": traffic,
            "flops_per_launch": main_res["flops_per_launch"],
            "avg_launch_us": g["avg_us"],
        },
        # every kernel timed, over a few extra steps after the timed region
        "kernels_avg_us": {k: round(v["avg_us"], 3) for k, v in main_res["kernels"].items()},
        "warmup_until_steady": main_res["warmup"],
        "final_mu": main_res["final_mu"],
        "other_modes": others,
        "plain_workload": plain,
        "small_solve": small,
        "equal_mu": equal,
        "batched": batched,
        "serving": serving,
        "serving_reachable_target": serving_reachable,
        "smooth_max": smooth,
        "optimiser_table2": table2,
        "miso_codebook": miso,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(wl, inputs.MEDIUM, inputs.SMALL, args.cpu_seconds, equal_frames)
        line["cpu_baseline"]["gpu_speedup"] = main_res["evals_per_s"] / line["cpu_baseline"]["value"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
