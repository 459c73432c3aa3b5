"""Random draws of the candidate search (oracle copy).

The paper starts from a random collection of unit vectors (Alg. 2 step 1) and
does not say how randomness is produced.  This is the reading used by both
sides of the project:

* generator: Philox4x32-10 (see ``philox``), key = (seed, stream_id);
* counter  : (block, candidate c, step t, tag), tag 0 = trust-region
  perturbation, tag 1 = random start (c = 0, t = 0 for the start);
* blocks   : column j of a d x N frame owns ceil(d/2) consecutive blocks,
  block = j * ceil(d/2) + q, and block q yields entries 2q and 2q + 1 of that
  column (for odd d the second entry of the last block is unused);
* uniforms : word w -> u = (w + 1/2) * 2^-32, strictly inside (0, 1);
* Gaussians: Box-Muller (Box and Muller, 1958) on (u0, u1) and (u2, u3):
  g0 = r cos(2 pi u1), g1 = r sin(2 pi u1) with r = sqrt(-2 ln u0), likewise g2, g3;
* complex  : z_{2q} = (g0 + i g1) / sqrt(2), z_{2q+1} = (g2 + i g3) / sqrt(2),
  so every entry is CN(0, 1) with E|z|^2 = 1.
"""

from __future__ import annotations

import math

import numpy as np

from .philox import philox4x32_10

TAG_PERTURB = 0
TAG_HAAR = 1

SQRT_HALF = math.sqrt(0.5)


def uniforms_from_words(words):
    """u = (w + 1/2) * 2^-32 in FP64 (exact for every 32-bit w)."""
    w = np.asarray(words, dtype=np.float64)
    return (w + 0.5) * (2.0 ** -32)


def box_muller(u0, u1):
    """One Box-Muller pair: (r cos(2 pi u1), r sin(2 pi u1)), r = sqrt(-2 ln u0)."""
    r = np.sqrt(-2.0 * np.log(u0))
    theta = 2.0 * np.pi * u1
    return r * np.cos(theta), r * np.sin(theta)


def complex_gaussian_frame(n, d, seed, stream_id, cand, t, tag):
    """The d x N matrix of CN(0,1) entries drawn for candidate(s) ``cand`` at step ``t``.

    ``cand`` may be an int or a 1-D array of candidate indices; the result has
    shape (d, n) or (len(cand), d, n).
    """
    n, d = int(n), int(d)
    scalar = np.ndim(cand) == 0
    cands = np.atleast_1d(np.asarray(cand, dtype=np.uint64))
    nb = (d + 1) // 2
    if n * nb >= 2 ** 32:
        raise ValueError("frame too large for the 32-bit block counter")
    blocks = np.arange(n * nb, dtype=np.uint64)  # block = j * nb + q
    C = cands.size
    ctr = np.empty((C, n * nb, 4), dtype=np.uint64)
    ctr[..., 0] = blocks[None, :]
    ctr[..., 1] = cands[:, None]
    ctr[..., 2] = np.uint64(t)
    ctr[..., 3] = np.uint64(tag)
    key = np.array([int(seed) & 0xFFFFFFFF, int(stream_id) & 0xFFFFFFFF], dtype=np.uint64)
    w = philox4x32_10(ctr, key)                       # (C, n*nb, 4)
    u = uniforms_from_words(w)
    g0, g1 = box_muller(u[..., 0], u[..., 1])
    g2, g3 = box_muller(u[..., 2], u[..., 3])
    za = (g0 + 1j * g1) * SQRT_HALF                   # entry 2q
    zb = (g2 + 1j * g3) * SQRT_HALF                   # entry 2q + 1
    z = np.stack([za, zb], axis=-1).reshape(C, n, nb * 2)[:, :, :d]   # (C, n, d)
    out = np.ascontiguousarray(np.transpose(z, (0, 2, 1)))            # (C, d, n)
    return out[0] if scalar else out
