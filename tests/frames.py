"""Frames with known coherence, built from their mathematical definitions.

Used as fixtures for the oracle's pins and for the GPU parity tests.  None of
these uses the candidate search.  Every frame is returned as a d x N complex
array whose columns are the vectors.
"""

from __future__ import annotations

import math

import numpy as np


def onb(d):
    """Orthonormal basis: N = d, coherence 0."""
    return np.eye(d, dtype=np.complex128)


def three_lines_in_plane():
    """Three real lines in R^2 at 60 degrees: coherence cos(60) = 1/2 (Welch-tight, N=3, d=2)."""
    th = np.array([0.0, math.pi / 3, 2 * math.pi / 3])
    return np.stack([np.cos(th), np.sin(th)]).astype(np.complex128)


def hopf_lift(points):
    """Map unit vectors n on S^2 to unit vectors in C^2 (the CP^1 <-> S^2
    correspondence mentioned in §I):  psi = (cos(a/2), e^{ib} sin(a/2)) for
    n = (sin a cos b, sin a sin b, cos a).  Then |<psi, psi'>|^2 = (1 + n.n')/2."""
    P = np.asarray(points, dtype=np.float64)
    P = P / np.linalg.norm(P, axis=1, keepdims=True)
    a = np.arccos(np.clip(P[:, 2], -1, 1))
    b = np.arctan2(P[:, 1], P[:, 0])
    return np.stack([np.cos(a / 2) + 0j, np.exp(1j * b) * np.sin(a / 2)])


def tetrahedron_c2():
    """Regular tetrahedron -> 4 lines in C^2 (the d=2 SIC): coherence 1/sqrt(3)."""
    return hopf_lift([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]])


def octahedron_c2():
    """Octahedron -> 6 lines in C^2 (3 mutually unbiased bases): coherence 1/sqrt(2)."""
    return hopf_lift([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]])


def icosahedron_c2():
    """Icosahedron vertices -> 12 lines in C^2: coherence sqrt((1 + 1/sqrt 5)/2)."""
    g = (1 + math.sqrt(5)) / 2
    pts = []
    for s1 in (1, -1):
        for s2 in (1, -1):
            pts += [[0, s1, s2 * g], [s1, s2 * g, 0], [s2 * g, 0, s1]]
    return hopf_lift(pts)


def simplex(d):
    """N = d + 1 vectors of the regular simplex in R^d: coherence 1/d.

    Centre the standard basis of R^{d+1}, then express it in an orthonormal
    basis of the sum-zero hyperplane (from a QR factorisation)."""
    E = np.eye(d + 1) - 1.0 / (d + 1)
    Q, _ = np.linalg.qr(E[:, :d])          # orthonormal basis of the column space (the hyperplane)
    V = Q.T @ E                             # coordinates, (d, d+1)
    return (V / np.linalg.norm(V, axis=0)).astype(np.complex128)


def weyl_heisenberg(fiducial):
    """All d^2 vectors X^a Z^b psi (shift X, clock Z with omega = e^{2 pi i/d})."""
    psi = np.asarray(fiducial, dtype=np.complex128)
    d = psi.size
    w = np.exp(2j * math.pi / d)
    cols = []
    for a in range(d):
        for b in range(d):
            v = np.roll(psi * w ** (b * np.arange(d)), a)
            cols.append(v)
    F = np.stack(cols, axis=1)
    return F / np.linalg.norm(F, axis=0)


def hesse_sic():
    """Hesse SIC: N = 9 lines in C^3, Weyl-Heisenberg orbit of (0, 1, -1)/sqrt 2;
    coherence 1/2 (Welch-tight) and Phi Phi^* = 3 I."""
    return weyl_heisenberg(np.array([0, 1, -1]) / math.sqrt(2))


def naimark_complement(Phi):
    """Gale dual / Naimark complement (§II): complete the rows of the scaled
    tight frame to a unitary; the remaining rows give N vectors in C^{N-d}."""
    from scipy.linalg import null_space
    d, N = Phi.shape
    B = null_space(np.conj(Phi))           # (N, N-d), columns orthogonal to the rows of Phi
    Psi = B.T
    return Psi / np.linalg.norm(Psi, axis=0)


def mub_frame(p):
    """All p + 1 mutually unbiased bases of C^p for an odd prime p (§V):
    the standard basis and the bases v_{a,b}[x] = omega^{a x^2 + b x}/sqrt p.
    N = p(p + 1), coherence 1/sqrt p (orthoplex- and Levenshtein-tight)."""
    w = np.exp(2j * math.pi / p)
    x = np.arange(p)
    cols = [np.eye(p, dtype=np.complex128)[:, i] for i in range(p)]
    for a in range(p):
        for b in range(p):
            cols.append(w ** ((a * x * x + b * x) % p) / math.sqrt(p))
    return np.stack(cols, axis=1)


def sic_numeric(d, seed=0):
    """A Welch-tight N = d^2 frame in C^d found numerically without the
    candidate search: minimise the frame potential sum_{j,k} |<phi_j,phi_k>|^4,
    whose minimum 2 N^2 / (d (d + 1)) is attained exactly by SICs (Welch's
    higher-order bound), then polish |G_jk|^2 = 1/(d + 1) by least squares."""
    from scipy.optimize import least_squares, minimize
    N = d * d
    rng = np.random.default_rng(seed)

    def unpack(x):
        Z = (x[: d * N] + 1j * x[d * N:]).reshape(d, N)
        return Z / np.linalg.norm(Z, axis=0)

    def potential(x):
        F = unpack(x)
        G = F.conj().T @ F
        return float(np.sum(np.abs(G) ** 4))

    best = None
    for attempt in range(20):
        x0 = rng.standard_normal(2 * d * N)
        r = minimize(potential, x0, method="L-BFGS-B", options={"maxiter": 5000, "gtol": 1e-14})
        if best is None or r.fun < best.fun:
            best = r
        if abs(r.fun - 2.0 * N * N / (d * (d + 1))) < 1e-6:
            break
    iu = np.triu_indices(N, 1)

    def resid(x):
        F = unpack(x)
        G = F.conj().T @ F
        return np.abs(G[iu]) ** 2 - 1.0 / (d + 1)

    r2 = least_squares(resid, best.x, xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=2000)
    return unpack(r2.x)


KNOWN = {
    # name: (builder, exact coherence)
    "onb4": (lambda: onb(4), 0.0),
    "three_lines": (three_lines_in_plane, 0.5),
    "tetrahedron": (tetrahedron_c2, 1 / math.sqrt(3)),
    "octahedron": (octahedron_c2, 1 / math.sqrt(2)),
    "icosahedron": (icosahedron_c2, math.sqrt((1 + 1 / math.sqrt(5)) / 2)),
    "simplex5": (lambda: simplex(5), 1 / 5),
    "hesse": (hesse_sic, 0.5),
    "naimark_hesse": (lambda: naimark_complement(hesse_sic()), 0.25),
    "mub3": (lambda: mub_frame(3), 1 / math.sqrt(3)),
    "mub5": (lambda: mub_frame(5), 1 / math.sqrt(5)),
}
