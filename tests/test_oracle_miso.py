"""Pins of the §III codebook quantiser and distortion oracle (CPU only).

Each pin is fixed by something other than the oracle's own formula: closed
forms of the distortion for one codeword and for an orthonormal basis
(Beta and exponential order statistics), the chordal distance written as the
distance between the projections onto the two lines, the identification of
lines in C^2 with points of the sphere S^2 (Bloch vectors, which §II
mentions) with a quadrature of the expected distortion of the octahedron
codebook, invariances and the tie and invalid-input rules.
"""

import math

import numpy as np
import pytest

import frames
import inputs
import oracle


def _mc_close(samples, expect, k=5.0):
    """|mean - expect| within k standard errors of the sample mean."""
    se = np.std(samples) / math.sqrt(samples.size)
    assert abs(np.mean(samples) - expect) <= k * se, (np.mean(samples), expect, se)


@pytest.mark.parametrize("d", [2, 4, 8, 33])
def test_single_codeword_closed_form(d):
    """One codeword: |<phi, h/|h|>|^2 ~ Beta(1, d - 1), so D = 1 - 1/d, and
    |<phi, h>|^2 ~ Exp(1), so the mean gain is 1."""
    phi = inputs.random_frame(1, d, seed=d)
    H = inputs.miso_channels(100000, d, seed=100 + d)
    index, gain, dist = oracle.quantize(phi, H)
    assert np.all(index == 0)
    _mc_close(dist, 1.0 - 1.0 / d)
    _mc_close(gain, 1.0)
    # the sample variance of the distortion against the Beta variance
    var = (d - 1) / (d * d * (d + 1))
    assert abs(np.var(dist) / var - 1.0) < 0.05


@pytest.mark.parametrize("d", [2, 3, 5, 8])
def test_orthonormal_basis_closed_form(d):
    """An orthonormal basis (rotated by a random unitary): |<e_i, h>|^2 are
    d i.i.d. Exp(1) variables, so the mean gain is E[max] = H_d (harmonic
    number) and, the normalised vector being uniform on the simplex, the mean
    of max / sum is H_d / d, so D = 1 - H_d / d."""
    Hd = sum(1.0 / k for k in range(1, d + 1))
    Q, _ = np.linalg.qr(inputs.random_frame(d, d, seed=7, scale_spread=False))
    H = inputs.miso_channels(120000, d, seed=3 * d)
    _, gain, dist = oracle.quantize(Q, H)
    _mc_close(dist, 1.0 - Hd / d)
    _mc_close(gain, Hd)


def _projection_distance_sq(x, y):
    """Chordal distance between the lines of x and y as the Frobenius distance
    of the rank-one projections: d_c^2 = |P_x - P_y|_F^2 / 2."""
    Px = np.outer(x, x.conj()) / np.vdot(x, x).real
    Py = np.outer(y, y.conj()) / np.vdot(y, y).real
    D = Px - Py
    return float(np.sum(np.abs(D) ** 2)) / 2.0


@pytest.mark.parametrize("n,d,seed", [(5, 3, 0), (9, 2, 1), (12, 4, 2), (3, 7, 3)])
def test_nearest_line_by_projection_distance(n, d, seed):
    """The quantiser picks the codeword at least chordal distance, and its
    distance is that minimum (the equivalence of the argmax and the argmin
    that §III states), checked by loops over the projection form."""
    C = inputs.random_frame(n, d, seed=seed)
    H = inputs.miso_channels(40, d, seed=seed + 50)
    index, gain, dist = oracle.quantize(C, H)
    for m in range(H.shape[1]):
        ds = [_projection_distance_sq(H[:, m], C[:, i]) for i in range(n)]
        best = int(np.argmin(ds))
        srt = sorted(ds)
        assert srt[1] - srt[0] > 1e-9           # random data: a unique minimum
        assert index[m] == best
        assert abs(dist[m] - ds[best]) <= 1e-12
        h2 = float(np.vdot(H[:, m], H[:, m]).real)
        assert abs(gain[m] - h2 * (1.0 - ds[best])) <= 1e-12 * h2


def _bloch(x):
    """Unit vector of S^2 for the line of x in C^2 (x x^* / |x|^2 = (I + b.sigma) / 2)."""
    x = x / np.linalg.norm(x)
    a, b = x[0], x[1]
    return np.array([2 * (np.conj(a) * b).real, 2 * (np.conj(a) * b).imag, abs(a) ** 2 - abs(b) ** 2])


def test_lines_in_c2_as_points_of_the_sphere():
    """Lines of C^2 are points of S^2, with |<x, y>|^2 = (1 + b_x . b_y) / 2 for
    unit x, y: the quantiser is the nearest point on the sphere.  For the
    octahedron codebook (the three mutually unbiased bases of C^2, Bloch
    vectors +-e_1, +-e_2, +-e_3) D = (1 - E max(|z_1|, |z_2|, |z_3|)) / 2 for
    z uniform on S^2, the expectation taken by quadrature."""
    s = 1 / math.sqrt(2)
    C = np.array([[1, 0], [0, 1], [s, s], [s, -s], [s, 1j * s], [s, -1j * s]], dtype=complex).T
    B = np.array([_bloch(C[:, i]) for i in range(6)])
    assert np.allclose(np.abs(B).sum(axis=1), 1.0)
    H = inputs.miso_channels(200000, 2, seed=9)
    index, gain, dist = oracle.quantize(C, H)
    for m in range(200):
        bh = _bloch(H[:, m])
        dots = B @ bh
        assert index[m] == int(np.argmax(dots))
        assert abs(dist[m] - (1 - dots.max()) / 2) <= 1e-12
    from scipy import integrate

    def f(phi, th):
        z = (math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), math.cos(th))
        return max(abs(z[0]), abs(z[1]), abs(z[2])) * math.sin(th) / (4 * math.pi)

    # eight octants are alike: integrate one (theta in [0, pi/2], phi in [0, pi/2]) and scale
    e_max, _ = integrate.dblquad(f, 0, math.pi / 2, 0, math.pi / 2, epsabs=1e-10)
    _mc_close(dist, (1 - 8 * e_max) / 2)


def test_invariances():
    """A common unitary on codebook and channels, and column scales and phases
    of the codebook, leave the quantiser unchanged."""
    n, d = 20, 4
    C = inputs.random_frame(n, d, seed=1)
    H = inputs.miso_channels(500, d, seed=2)
    i0, g0, d0 = oracle.quantize(C, H)
    U, _ = np.linalg.qr(inputs.random_frame(d, d, seed=3, scale_spread=False))
    i1, g1, d1 = oracle.quantize(U @ C, U @ H)
    assert np.array_equal(i0, i1) and np.allclose(g0, g1, rtol=1e-12) and np.allclose(d0, d1, atol=1e-12)
    ph = np.exp(2j * np.pi * np.random.default_rng(4).random(n)) * (0.5 + np.arange(n))
    i2, g2, d2 = oracle.quantize(C * ph[None, :], H)
    assert np.array_equal(i0, i2) and np.allclose(g0, g2, rtol=1e-12) and np.allclose(d0, d2, atol=1e-12)


def test_ties_go_to_the_lowest_index_and_codewords_quantise_to_themselves():
    d = 3
    C = inputs.random_frame(4, d, seed=5)
    C = np.concatenate([C, C[:, 1:2] * (2.0 * np.exp(0.7j))], axis=1)   # codeword 4 = line of codeword 1
    H = C[:, [1, 4, 2]] * np.array([3.0, 0.5j, -1.0])[None, :]
    index, gain, dist = oracle.quantize(C, H)
    assert index[2] == 2 and abs(dist[2]) <= 1e-15
    assert abs(dist[0]) <= 1e-15 and abs(dist[1]) <= 1e-15
    assert index[0] in (1, 4) and index[1] in (1, 4)
    # an exact tie: a channel orthogonal to every codeword but e_0, e_1, whose
    # inner products with both have equal modulus
    E = np.eye(3, dtype=complex)
    idx, g, _ = oracle.quantize(E, np.array([[1.0], [1.0j], [0.0]]))
    assert idx[0] == 0 and g[0] == 1.0


def test_invalid_codeword_and_zero_channel():
    C = inputs.random_frame(5, 3, seed=6)
    C[:, 2] = 0
    index, gain, dist = oracle.quantize(C, inputs.miso_channels(7, 3, seed=1))
    assert np.all(index == -1) and np.all(np.isnan(gain)) and np.all(np.isnan(dist))
    C = inputs.random_frame(5, 3, seed=6)
    H = inputs.miso_channels(3, 3, seed=1)
    H[:, 1] = 0
    index, gain, dist = oracle.quantize(C, H)
    assert index[1] == 0 and gain[1] == 0 and np.isnan(dist[1]) and np.isfinite(dist[[0, 2]]).all()
    ref_i, ref_g, ref_d = index.copy(), gain.copy(), dist.copy()
    H[1, 0] = np.inf
    H[0, 2] = np.nan
    H[:, 1] = 1e200                      # finite entries whose squared norm overflows
    index, gain, dist = oracle.quantize(C, H)
    assert np.all(index == -1) and np.all(np.isnan(gain)) and np.all(np.isnan(dist))
    H = inputs.miso_channels(3, 3, seed=1)
    H[2, 1] = -np.inf
    index, gain, dist = oracle.quantize(C, H)
    assert index[1] == -1 and np.isnan(gain[1]) and np.isnan(dist[1])
    assert np.array_equal(index[[0, 2]], ref_i[[0, 2]]) and np.array_equal(gain[[0, 2]], ref_g[[0, 2]])


def test_distortion_falls_with_better_packings():
    """Codebooks that pack lines well quantise better: at N = 4 in C^2 the SIC
    (tetrahedron, coherence 1/sqrt 3) has lower distortion than four random
    lines on average, and any codebook stays below the one-codeword value."""
    H = inputs.miso_channels(100000, 2, seed=11)
    sic = frames.tetrahedron_c2()
    assert abs(oracle.coherence(sic) - 1 / math.sqrt(3)) < 1e-12
    D_sic, _ = oracle.distortion(sic, H)
    Ds = [oracle.distortion(inputs.random_frame(4, 2, seed=s), H)[0] for s in range(20)]
    assert D_sic < np.mean(Ds) and D_sic <= min(Ds) + 3e-3
    assert max(Ds) < 0.5
