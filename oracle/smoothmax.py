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


def smooth_max_grad(Y, delta):
    """Real gradient of F_{s,delta} over x = |G_jk|^2 (j < k) with respect to
    the unconstrained frame Y (§IV: the columns of Y are normalised inside
    the objective), returned as a complex d x N matrix g with
    dF = sum Re(conj(g) * dY), i.e. g = 2 dF/d conj(Y).

    The steps follow the chain of definitions:
      w_jk = dF/dx_jk = exp((x_jk - s)/delta) / sum exp((x - s)/delta)
             (the shift s cancels; w is symmetric, zero on the diagonal);
      dx_jk/d conj(phi_k) = G_jk phi_j and dx_jk/d conj(phi_j) = conj(G_jk) phi_k,
      so D = dF/d conj(Phi) = Phi (W o G);
      phi_k = y_k / r_k gives dF/d conj(y_k) = (D_k - phi_k Re(phi_k^H D_k)) / r_k.
    Returns None for a frame with a zero or non-finite column."""
    Y = np.asarray(Y, dtype=np.complex128)
    Phi, norms = normalize_columns(Y)
    if not np.all(np.isfinite(norms) & (norms > 0.0)):
        return None
    G = gram(Phi)
    N = G.shape[0]
    X = G.real * G.real + G.imag * G.imag
    iu = np.triu_indices(N, k=1)
    s = float(np.max(X[iu]))
    np.fill_diagonal(X, s)            # the diagonal is not a pair: zeroed below
    E = np.exp((X - s) / delta)
    np.fill_diagonal(E, 0.0)
    total = math.fsum(E[iu].tolist())
    W = E / total                     # symmetric, both triangles carry w_jk
    D = Phi @ (W * G)
    c = np.sum((Phi.conj() * D).real, axis=0)
    return 2.0 * (D - Phi * c[None, :]) / norms[None, :]


def smooth_max_hess_vec(Y, V, delta):
    """Exact Hessian-vector product of F_{s,delta} over x = |G_jk|^2 (j < k)
    with respect to the unconstrained frame Y, in the direction V: the
    derivative d/dt of ``smooth_max_grad(Y + t V)`` at t = 0 (B_k of Alg. 1
    in §IV is the Hessian of the objective).  Same convention as the
    gradient: the result H with <U, H> = sum Re(conj(U) H) equals the second
    derivative of F along U and V.

    Forward differentiation of every line of the gradient's chain:
      r_k = |y_k|, phi_k = y_k / r_k:
        dr_k = Re(phi_k^H v_k),  dphi_k = (v_k - phi_k dr_k) / r_k;
      G = Phi^H Phi:  dG = dPhi^H Phi + Phi^H dPhi;
      x_jk = |G_jk|^2:  dx_jk = 2 Re(conj(G_jk) dG_jk);
      w_jk = e_jk / sum_{l<m} e_lm, e = exp((x - s) / delta) (the shift s
        cancels, so its own derivative does not enter):
        dw_jk = w_jk (dx_jk - sigma) / delta,  sigma = sum_{l<m} w_lm dx_lm;
      D = Phi (W o G):  dD = dPhi (W o G) + Phi (dW o G + W o dG);
      c_k = Re(phi_k^H D_k):  dc_k = Re(dphi_k^H D_k + phi_k^H dD_k);
      g_k = 2 (D_k - phi_k c_k) / r_k:
        dg_k = 2 (dD_k - dphi_k c_k - phi_k dc_k) / r_k - g_k dr_k / r_k.
    Returns None for a frame with a zero or non-finite column."""
    Y = np.asarray(Y, dtype=np.complex128)
    V = np.asarray(V, dtype=np.complex128)
    Phi, norms = normalize_columns(Y)
    if not np.all(np.isfinite(norms) & (norms > 0.0)):
        return None
    N = Phi.shape[1]
    dr = np.sum((Phi.conj() * V).real, axis=0)
    dPhi = (V - Phi * dr[None, :]) / norms[None, :]
    G = gram(Phi)
    dG = dPhi.conj().T @ Phi + Phi.conj().T @ dPhi
    X = G.real * G.real + G.imag * G.imag
    dX = 2.0 * (G.conj() * dG).real
    iu = np.triu_indices(N, k=1)
    s = float(np.max(X[iu]))
    np.fill_diagonal(X, s)
    E = np.exp((X - s) / delta)
    np.fill_diagonal(E, 0.0)
    total = math.fsum(E[iu].tolist())
    W = E / total
    sigma = math.fsum((W[iu] * dX[iu]).tolist())
    dW = W * (dX - sigma) / delta
    np.fill_diagonal(dW, 0.0)
    D = Phi @ (W * G)
    dD = dPhi @ (W * G) + Phi @ (dW * G + W * dG)
    c = np.sum((Phi.conj() * D).real, axis=0)
    dc = np.sum((dPhi.conj() * D).real, axis=0) + np.sum((Phi.conj() * dD).real, axis=0)
    g = 2.0 * (D - Phi * c[None, :]) / norms[None, :]
    return 2.0 * (dD - dPhi * c[None, :] - Phi * dc[None, :]) / norms[None, :] - g * (dr / norms)[None, :]
