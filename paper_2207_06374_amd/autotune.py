"""Tile autotuners.

Batched form: the batched kernel processes each candidate with 1, 2 or 4
wavefronts (``waves_per_item``).  The choice changes only speed, never
results (each pair is computed by the same code whatever the split).  This
module times every feasible choice on homogeneous batches of one (d, N) class
and keeps the fastest per class in a JSON table; ``Batch`` consults the table
for instances that do not fix ``waves_per_item`` themselves.

BF16 screen (single searches, solves and the serving engine): the tile form
(blocks of 256 frame rows, 64 per wavefront, for 2d <= 128; or of 128 rows,
32 per wavefront) and the run length (column tiles of 128 a block sweeps
after loading its rows) are timed per (K steps, N) class with whole steps of
64 candidates, and the fastest go to ``screen_tiles.json``, which the binding
installs in the library when it loads it.  Every choice gives the same
screened values (each pair's product is the same MFMA sequence), so results
never change.

Run on the GPU:  python -m paper_2207_06374_amd.autotune [--out PATH]
                 python -m paper_2207_06374_amd.autotune --screen [--screen-out PATH]
"""

from __future__ import annotations

import argparse
import json
import os
import time

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_tiles.json")
N_BUCKETS = (16, 32, 64, 128, 256)
LDS_WORDS = 9216   # LDS words of a step block's candidate copies


def ldk(d):
    """LDS words per column of a candidate's split copy: hi and lo planes of
    2d reals padded to a multiple of 8, plus 16 bytes."""
    return (2 * d + 7) // 8 * 8 + 4


def feasible(n, d):
    return [w for w in (1, 2, 4) if n * ldk(d) * (4 // w) <= LDS_WORDS]


def classes(d_lo=3, d_hi=16):
    """(d, n_max) classes covering N in [d + 1, min(d^2, 256)]."""
    out = []
    for d in range(d_lo, d_hi + 1):
        n_hi = min(d * d, 256)
        lo = d + 1
        for b in N_BUCKETS:
            if b >= lo:
                out.append((d, min(b, n_hi)))
            if b >= n_hi:
                break
    return out


def load_table(path=TABLE_PATH):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def choose(table, n, d):
    """waves_per_item for an (n, d) instance: the entry of the same d with the
    smallest n_max >= n; 0 (library default) when the table has none."""
    if not table:
        return 0
    best = None
    for e in table.get("entries", []):
        if e["d"] == d and e["n_max"] >= n and (best is None or e["n_max"] < best["n_max"]):
            best = e
    if best is None or best["wpi"] not in feasible(n, d):
        return 0
    return int(best["wpi"])


def time_class(lib, torch, d, n, wpi, count=128, candidates=64, steps=6):
    specs = [{"n": n, "d": d, "seed": 0, "stream_id": k, "max_steps": 10 ** 9, "waves_per_item": wpi}
             for k in range(count)]
    b = lib.Batch(specs, candidates=candidates).init()
    b.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e6


def autotune(out=TABLE_PATH, candidates=64, count=128, steps=6, verbose=True):
    import torch

    import paper_2207_06374_amd as lib
    entries = []
    for d, n in classes():
        times = {w: time_class(lib, torch, d, n, w, count, candidates, steps) for w in feasible(n, d)}
        w = min(times, key=times.get)
        entries.append({"d": d, "n_max": n, "wpi": w, "us_per_step": {str(k): round(v, 2) for k, v in times.items()}})
        if verbose:
            print(f"d={d:2d} n<={n:3d}: " + "  ".join(f"wpi={k}: {v:8.1f} us" for k, v in times.items())
                  + f"  -> {w}", flush=True)
    table = {"version": 1, "candidates": candidates, "instances_per_class": count, "entries": entries}
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
    return table


SCREEN_TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "screen_tiles.json")
# (d, n_max) classes: the serving mix (d in {8, 16, 32, 64, 128}, N in
# [2d, 8d]) in N buckets, and the throughput shape N = 4096, d = 64
SCREEN_CLASSES = ((16, 64), (16, 128), (32, 128), (32, 256), (64, 128), (64, 256), (64, 512), (64, 4096),
                  (128, 256), (128, 512), (128, 1024))
SCREEN_SEGS = (1, 2, 3, 4, 6, 8, 12, 16)


def screen_options(d):
    ks = (2 * d + 31) // 32
    forms = (0, 1) if ks <= 4 else (1,)
    return [(f, g) for f in forms for g in SCREEN_SEGS]


def time_screen(lib, torch, n, d, form, seg, candidates=64, steps=20, reps=3):
    """Microseconds per whole BF16-screen step (64 candidates) with this tile
    choice installed for (ks, n)."""
    from . import _abi
    ks = (2 * d + 31) // 32
    _abi.set_screen_tiles([{"ks": ks, "n_max": n, "form": form, "seg": seg}])
    s = lib.Solver(n, d, candidates=candidates, mode="bf16", radius0=0.05, max_steps=10 ** 6, seed=0)
    s.init_haar()
    for _ in range(3):
        s.step(with_report=False)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        for _ in range(steps):
            s.step(with_report=False)
        torch.cuda.synchronize()
        best = min(best, (time.perf_counter() - t0) / steps * 1e6)
    return best


def autotune_screen(out=SCREEN_TABLE_PATH, candidates=64, steps=20, verbose=True):
    import torch

    import paper_2207_06374_amd as lib
    from . import _abi
    entries = []
    try:
        for d, n in SCREEN_CLASSES:
            times = {(f, g): time_screen(lib, torch, n, d, f, g, candidates, steps) for f, g in screen_options(d)}
            f, g = min(times, key=times.get)
            default = (0, 6) if (2 * d + 31) // 32 <= 4 else (1, 8)
            entries.append({"ks": (2 * d + 31) // 32, "n_max": n, "d": d, "form": f, "seg": g,
                            "us_per_step": round(times[(f, g)], 2), "default_us_per_step": round(times[default], 2)})
            if verbose:
                print(f"d={d:3d} n<={n:4d}: best form {f} seg {g:2d} {times[(f, g)]:9.1f} us/step "
                      f"(default {times[default]:9.1f})", flush=True)
    finally:
        _abi.set_screen_tiles([])
    table = {"version": 1, "candidates": candidates, "entries": entries}
    with open(out, "w") as f:
        json.dump(table, f, indent=1)
    _abi.set_screen_tiles(entries)
    return table


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--count", type=int, default=128)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--screen", action="store_true", help="tune the BF16 screen's tiles instead")
    ap.add_argument("--screen-out", default=SCREEN_TABLE_PATH)
    args = ap.parse_args()
    if args.screen:
        autotune_screen(args.screen_out)
    else:
        autotune(args.out, count=args.count, steps=args.steps)
