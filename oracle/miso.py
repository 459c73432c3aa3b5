"""Beamforming-codebook evaluation of §III, the MISO application (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

The model of §III: d transmit antennas, one receive antenna, a channel h
with i.i.d. CN(0, 1) entries.  Transmitter and receiver share a codebook of
N unit vectors phi_1..phi_N; the receiver picks the index that maximises
|<phi_i, h>|^2 and feeds it back, and the received SNR is E_s / sigma times
that maximum.  Seen as a quantiser, Q_Phi maps the line of h to that codeword,
which is also the codeword at least chordal distance from it, and the
distortion of the codebook is the expected squared chordal distance between a
uniformly distributed line and its quantisation.  The line of a CN(0, I_d)
vector is uniformly distributed on CP^{d-1}, so averaging over drawn channels
estimates it.

Chordal distance between the lines of unit vectors x, y (§II):
d_c(x, y)^2 = 1 - |<x, y>|^2.  Inner products are <x, y> = sum conj(x_k) y_k.
"""

from __future__ import annotations

import numpy as np

from .coherence import normalize_columns


def quantize(codebook, H):
    """Quantise every channel column of H (d x M) with the codebook (d x N,
    columns normalised here, as §III takes unit codewords).

    Returns ``(index, gain, dist)``, each of length M:
    index[m] = argmax_i |<phi_i, h_m>|^2 (the first of equal maxima),
    gain[m]  = that maximum (the SNR in units of E_s / sigma),
    dist[m]  = d_c^2(h_m / |h_m|, phi_index) = 1 - gain[m] / |h_m|^2.
    A codeword of zero or non-finite norm makes the codebook invalid: every
    index is -1 and every gain and distance NaN.  A channel whose squared
    norm is not finite (a non-finite entry, or overflow) gets index -1 and
    NaN gain and distance; a zero channel has gain 0 at index 0 and a NaN
    distance (its line is undefined).  The paper draws channels from a
    Gaussian and fixes none of these cases.
    """
    H = np.asarray(H, dtype=np.complex128)
    M = H.shape[1]
    Phi, norms = normalize_columns(codebook)
    if not np.all(np.isfinite(norms) & (norms > 0.0)):
        return np.full(M, -1, dtype=np.int32), np.full(M, np.nan), np.full(M, np.nan)
    with np.errstate(over="ignore", invalid="ignore"):
        G = Phi.conj().T @ H                      # G[i, m] = <phi_i, h_m>
        P = G.real * G.real + G.imag * G.imag     # |<phi_i, h_m>|^2
        h2 = np.sum(H.real * H.real + H.imag * H.imag, axis=0)
    bad = ~np.isfinite(h2)
    P[:, bad] = 0.0
    index = np.argmax(P, axis=0).astype(np.int32)   # numpy returns the first maximum
    gain = P[index, np.arange(M)]
    with np.errstate(invalid="ignore", divide="ignore"):
        dist = 1.0 - gain / h2
    index[bad] = -1
    gain[bad] = np.nan
    dist[bad] = np.nan
    return index, gain, dist


def distortion(codebook, H):
    """Monte-Carlo estimates over the channels of H: (mean squared chordal
    distance of the quantiser, i.e. the distortion D(Phi); mean of the
    maximal |<phi_i, h>|^2, i.e. the mean SNR gain in units of E_s / sigma)."""
    _, gain, dist = quantize(codebook, H)
    return float(np.mean(dist)), float(np.mean(gain))
