"""Coherence of a frame and the lower bounds the paper quotes (oracle, FP64).

A frame is a d x N complex matrix whose column j is the vector phi_j (§II
represents a frame this way).  The coherence (§I) is the largest modulus of an
off-diagonal entry of the Gram matrix Phi^* Phi of the unit-normalised
columns; by symmetry only the strictly upper triangle j < k is needed (§IV,
description of the variable x).
"""

from __future__ import annotations

import math

import numpy as np


def normalize_columns(Y):
    """Divide every column of ``Y`` by its Euclidean norm (§IV remark on the
    unconstrained formulation: each column is divided by its norm).

    Returns ``(Phi, norms)``.  A column whose norm is zero or not finite cannot
    be normalised; its entries come back as NaN and the caller decides what
    that means (the candidate path marks such a candidate invalid).
    """
    Y = np.asarray(Y, dtype=np.complex128)
    norms = np.sqrt(np.sum(Y.real * Y.real + Y.imag * Y.imag, axis=0))
    bad = ~(np.isfinite(norms) & (norms > 0.0))
    safe = np.where(bad, 1.0, norms)
    Phi = Y / safe[None, :]
    if bad.any():
        Phi[:, bad] = np.nan
    return Phi, norms


def gram(Phi):
    """Gram matrix G = Phi^* Phi, G[j, k] = <phi_j, phi_k> = sum_i conj(Phi[i, j]) Phi[i, k] (§I)."""
    Phi = np.asarray(Phi, dtype=np.complex128)
    return Phi.conj().T @ Phi


def coherence_sq_upper(Phi):
    """max_{j<k} |G[j,k]|^2 for an already-normalised frame (the squared
    coherence; the paper's objective is stated on squared moduli in §IV).
    Uses a library matmul for G and takes the strict upper triangle."""
    G = gram(Phi)
    N = G.shape[0]
    if N < 2:
        raise ValueError("coherence needs at least two vectors")
    iu = np.triu_indices(N, k=1)
    g = G[iu]
    return float(np.max(g.real * g.real + g.imag * g.imag))


def coherence(Phi, normalize=True):
    """mu(Phi) = max_{j != k} |<phi_j, phi_k>| of the column-normalised frame (§I).

    A frame with a zero or non-finite column has no coherence; this returns
    +inf for it (the convention the candidate search uses for an invalid
    candidate).
    """
    Phi = np.asarray(Phi, dtype=np.complex128)
    if normalize:
        Phi, norms = normalize_columns(Phi)
        if not np.all(np.isfinite(norms) & (norms > 0.0)):
            return math.inf
    G = gram(Phi)
    N = G.shape[0]
    if N < 2:
        raise ValueError("coherence needs at least two vectors")
    iu = np.triu_indices(N, k=1)
    return float(np.max(np.abs(G[iu])))


def coherence_pair(Phi):
    """A pair attaining the coherence: (mu, j, k) with j < k and
    |<phi_j, phi_k>| = mu, the first such pair in the order j * N + k (the
    pair is not unique in general; the value is).  A zero or non-finite
    column gives (inf, -1, -1)."""
    Phi, norms = normalize_columns(Phi)
    if not np.all(np.isfinite(norms) & (norms > 0.0)):
        return math.inf, -1, -1
    G = gram(Phi)
    N = G.shape[0]
    if N < 2:
        raise ValueError("coherence needs at least two vectors")
    iu = np.triu_indices(N, k=1)          # row-major order: increasing j * N + k
    g = G[iu]
    q = int(np.argmax(g.real * g.real + g.imag * g.imag))
    return float(abs(g[q])), int(iu[0][q]), int(iu[1][q])


def coherence_bruteforce(Phi):
    """The same definition written as explicit loops over pairs j < k, with
    each inner product summed term by term.  For tiny frames only."""
    Phi = np.asarray(Phi, dtype=np.complex128)
    d, N = Phi.shape
    cols = []
    for j in range(N):
        s = 0.0
        for i in range(d):
            z = complex(Phi[i, j])
            s += z.real * z.real + z.imag * z.imag
        nrm = math.sqrt(s)
        cols.append([complex(Phi[i, j]) / nrm for i in range(d)])
    best = 0.0
    for j in range(N):
        for k in range(j + 1, N):
            acc = 0j
            for i in range(d):
                acc += cols[j][i].conjugate() * cols[k][i]
            best = max(best, abs(acc))
    return best


def welch_bound(N, d):
    """Welch bound sqrt((N - d) / (d (N - 1))) (§II).  For N <= d the bound is
    read as 0 (an orthonormal set exists); N >= 2 is required."""
    if N < 2 or d < 1:
        raise ValueError("Welch bound needs N >= 2 and d >= 1")
    return math.sqrt(max(0.0, (N - d) / (d * (N - 1))))


def orthoplex_bound(N, d):
    """Orthoplex bound 1/sqrt(d), valid when N > d^2 (§V, Proposition on the
    orthoplex and Levenshtein bounds).  Returns 0 when it does not apply."""
    if N <= d * d:
        return 0.0
    return 1.0 / math.sqrt(d)


def levenshtein_bound(N, d):
    """Levenshtein bound sqrt((2N - d(d+1)) / ((N - d)(d+1))), valid when
    N > d^2 (§V, same Proposition; the paper writes the frame size as n).
    Returns 0 when it does not apply."""
    if N <= d * d:
        return 0.0
    return math.sqrt((2.0 * N - d * (d + 1)) / ((N - d) * (d + 1.0)))


def lower_bound(N, d):
    """The largest of the three lower bounds above for (N, d)."""
    return max(welch_bound(N, d), orthoplex_bound(N, d), levenshtein_bound(N, d))
