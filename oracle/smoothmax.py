"""Smooth maximum of section IV (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's optimiser works on a smooth stand-in for the maximum of the
strict-upper-triangle moduli of the Gram matrix of the column-normalised
frame: the shifted log-sum-exp

    F_{s,delta}(x) = s + delta * log( sum_i exp((x_i - s) / delta) ),
    s = max_i x_i,  delta > 0,

over the n = N(N-1)/2 entries x of that triangle (§IV, definition of the
maximum approximation and of the variable x).  Its Proposition bounds it by
s <= F <= s + delta * log(n).  The method statement of §IV applies it to
squared moduli while the description of x speaks of moduli; both readings
are provided (``squared``).  The sum is exact-rounded (math.fsum), so the
only rounding is in each x_i, each exp and the final log.
"""

from __future__ import annotations

import math

import numpy as np

from .coherence import gram, normalize_columns


def upper_values(Phi, squared=True):
    """x_i: |G_jk|^2 (or |G_jk|) for j < k of the column-normalised frame,
    row by row.  Returns None for a frame with a zero or non-finite column."""
    Phi, norms = normalize_columns(Phi)
    if not np.all(np.isfinite(norms) & (norms > 0.0)):
        return None
    G = gram(Phi)
    N = G.shape[0]
    if N < 2:
        raise ValueError("the smooth maximum needs at least two vectors")
    iu = np.triu_indices(N, k=1)
    g = G[iu]
    m = g.real * g.real + g.imag * g.imag
    return m if squared else np.sqrt(m)


def smooth_max_of_values(x, delta):
    """(s, F_{s,delta}(x)) for a vector of values x (§IV definition)."""
    if not (delta > 0.0) or not math.isfinite(delta):
        raise ValueError("delta must be finite and > 0")
    x = np.asarray(x, dtype=np.float64)
    s = float(np.max(x))
    total = math.fsum(np.exp((x - s) / delta).tolist())
    return s, s + delta * math.log(total)


def smooth_max(Phi, delta, squared=True):
    """(s, F_{s,delta}) of a frame (columns normalised first).  A frame with a
    zero or non-finite column gives (+inf, +inf)."""
    x = upper_values(Phi, squared)
    if x is None:
        return math.inf, math.inf
    return smooth_max_of_values(x, delta)


def smooth_max_bruteforce(Phi, delta, squared=True):
    """The same definition with explicit loops over pairs j < k and
    term-by-term sums (tiny frames only)."""
    Phi = np.asarray(Phi, dtype=np.complex128)
    d, N = Phi.shape
    cols = []
    for j in range(N):
        nrm = math.sqrt(sum(abs(complex(Phi[i, j])) ** 2 for i in range(d)))
        cols.append([complex(Phi[i, j]) / nrm for i in range(d)])
    xs = []
    for j in range(N):
        for k in range(j + 1, N):
            acc = 0j
            for i in range(d):
                acc += cols[j][i].conjugate() * cols[k][i]
            m = acc.real * acc.real + acc.imag * acc.imag
            xs.append(m if squared else math.sqrt(m))
    s = max(xs)
    return s, s + delta * math.log(math.fsum(math.exp((v - s) / delta) for v in xs))
