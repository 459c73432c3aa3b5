"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds no arithmetic of the method (no normalisation, no Gram, no
coherence, no candidate generation): it only draws raw arrays and workload
descriptions from numpy's seeded generators, so both the HIP path and the
oracle can be fed identical inputs.

Workloads (synthetic stand-ins for the paper's random-start experiments; the
paper runs on random unit vectors only and uses no dataset):

* ``SMALL``    N=16 vectors in C^4, 64 candidates per step, radius 0.1, 2000 steps;
* ``MEDIUM``   N=1024 in C^32, 256 candidates, radius 0.05, 5000 steps;
* ``LARGE``    N=4096 in C^64, 128 candidates, radius 0.05 (the throughput
  workload; bfloat16 screen with the top 8 re-evaluated in FP64);
* ``batched_instances``  512 independent (d, N) with d uniform in {3..16} and
  N uniform in [d+1, d^2], 64 candidates each;
* ``miso_channels``      CN(0, I_d) channel vectors for the codebook
  evaluation of §III;
* ``serving_requests``   Poisson arrivals (mean gap 5 ms), d in
  {8, 16, 32, 64, 128}, N uniform in [2d, 8d].
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: int
    d: int
    candidates: int
    radius0: float
    steps: int
    seed: int = 0
    stream_id: int = 0


SMALL = Workload("N=16,d=4,C=64", 16, 4, 64, 0.1, 2000)
MEDIUM = Workload("N=1024,d=32,C=256", 1024, 32, 256, 0.05, 5000)
LARGE = Workload("N=4096,d=64,C=128", 4096, 64, 128, 0.05, 5000)


def random_frame(n, d, seed, scale_spread=True):
    """A d x N complex matrix of i.i.d. CN(0,1) entries, columns optionally
    scaled by factors in [0.25, 4) so that normalisation is exercised.
    Returned as a (d, n) complex128 numpy array."""
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((d, n)) + 1j * rng.standard_normal((d, n))) * np.sqrt(0.5)
    if scale_spread:
        z = z * (0.25 * 16.0 ** rng.random(n))[None, :]
    return z


def random_perturbation(n, d, count, seed):
    """``count`` d x N complex Gaussian matrices (shape (count, d, n)), for
    steps driven by explicit perturbations instead of the generator."""
    rng = np.random.default_rng(seed)
    shape = (count, d, n)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * np.sqrt(0.5)


def batched_instances(count=512, seed=0, d_lo=3, d_hi=16):
    """(d_i, N_i) for the batched workload: d uniform in {d_lo..d_hi}, N uniform
    in [d+1, d^2]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        d = int(rng.integers(d_lo, d_hi + 1))
        n = int(rng.integers(d + 1, d * d + 1))
        out.append((d, n))
    return out


def serving_requests(count, seed=1, mean_gap_s=0.005, dims=(8, 16, 32, 64, 128)):
    """Request stream for the serving workload: list of dicts with arrival
    time (s), d, N (uniform in [2d, 8d]) and seed (= request id)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(mean_gap_s))
        d = int(dims[int(rng.integers(0, len(dims)))])
        n = int(rng.integers(2 * d, 8 * d + 1))
        out.append({"id": i, "arrival": t, "d": d, "n": n, "seed": i})
    return out


def miso_channels(m, d, seed):
    """``m`` channel vectors of the MISO model (§III): a (d, m) complex128
    array whose entries are i.i.d. CN(0, 1) (real and imaginary parts
    N(0, 1/2))."""
    return random_frame(m, d, seed, scale_spread=False)
