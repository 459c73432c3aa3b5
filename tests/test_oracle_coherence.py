"""Pins for the oracle's coherence and bounds (CPU only).

Each check ties the oracle to something other than its own formula: explicit
pairwise loops, frames whose coherence is known in closed form, the values
printed in Table II, the bounds of §II and §V, and invariances of |<.,.>|.
"""

import math

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import frames
import inputs
import oracle
from conftest import golden_path


@pytest.mark.parametrize("n,d,seed", [(2, 1, 0), (3, 2, 1), (5, 2, 2), (7, 3, 3), (12, 5, 4), (9, 4, 5)])
def test_vectorised_matches_bruteforce(n, d, seed):
    F = inputs.random_frame(n, d, seed)
    assert abs(oracle.coherence(F) - oracle.coherence_bruteforce(F)) <= 1e-15


@pytest.mark.parametrize("name", sorted(frames.KNOWN))
def test_known_optima(name):
    build, mu = frames.KNOWN[name]
    F = build()
    assert abs(oracle.coherence(F) - mu) <= 1e-14
    # the squared form agrees with the modulus form
    Fn, _ = oracle.normalize_columns(F)
    assert abs(math.sqrt(oracle.coherence_sq_upper(Fn)) - mu) <= 1e-14


@pytest.mark.parametrize("name,welch_tight", [("three_lines", True), ("tetrahedron", True), ("simplex5", True),
                                              ("hesse", True), ("naimark_hesse", True)])
def test_welch_equality_at_etfs(name, welch_tight):
    F = frames.KNOWN[name][0]()
    d, N = F.shape
    assert abs(oracle.coherence(F) - oracle.welch_bound(N, d)) <= 1e-14


def test_hesse_is_tight_frame():
    F = frames.hesse_sic()
    assert np.allclose(F @ F.conj().T, 3 * np.eye(3), atol=1e-14)


def test_numeric_sic_d4_is_welch_tight():
    F = frames.sic_numeric(4)
    assert F.shape == (4, 16)
    assert abs(oracle.coherence(F) - math.sqrt(0.2)) <= 1e-12
    assert abs(oracle.welch_bound(16, 4) - math.sqrt(0.2)) <= 1e-16
    assert np.allclose(F @ F.conj().T, 4 * np.eye(4), atol=1e-10)


@pytest.mark.parametrize("p", [3, 5])
def test_mub_attains_orthoplex_and_levenshtein(p):
    F = frames.mub_frame(p)
    d, N = F.shape
    assert N == p * (p + 1) and N > d * d
    mu = oracle.coherence(F)
    assert abs(mu - oracle.orthoplex_bound(N, d)) <= 1e-14
    assert abs(mu - oracle.levenshtein_bound(N, d)) <= 1e-14
    # removing up to d-1 points keeps coherence 1/sqrt(d) (§V: N=(d+1)d-j optimal)
    assert abs(oracle.coherence(F[:, : N - (d - 1)]) - mu) <= 1e-14


def test_octahedron_is_orthoplex_tight():
    F = frames.octahedron_c2()
    assert abs(oracle.coherence(F) - oracle.orthoplex_bound(6, 2)) <= 1e-15
    assert abs(oracle.coherence(F[:, :5]) - 1 / math.sqrt(2)) <= 1e-15


def test_d1_all_parallel():
    F = inputs.random_frame(5, 1, 7)
    assert abs(oracle.coherence(F) - 1.0) <= 1e-15
    assert oracle.welch_bound(5, 1) == 1.0


def test_table2_sic_values_are_welch_values():
    rows = [l.split() for l in open(golden_path("table2_trstmi_mu.txt")) if l.strip() and not l.startswith("#")]
    for d, N, mu in rows:
        d, N, mu = int(d), int(N), float(mu)
        w = oracle.welch_bound(N, d)
        assert w <= mu + 1e-12                  # every printed coherence respects Welch
        if d <= 7:                              # printed value is 1/sqrt(d+1) rounded up
            assert mu - 1e-4 - 1e-12 <= w <= mu
            assert abs(w - 1 / math.sqrt(d + 1)) <= 1e-15
    # the closed-form / numeric SICs we can build reach the printed values
    assert oracle.coherence(frames.tetrahedron_c2()) <= 0.5774
    assert oracle.coherence(frames.hesse_sic()) <= 0.5001
    assert oracle.coherence(frames.sic_numeric(4)) <= 0.4473


def test_bounds_closed_forms():
    assert oracle.welch_bound(4, 4) == 0.0
    assert oracle.welch_bound(3, 5) == 0.0            # N <= d read as 0
    assert abs(oracle.welch_bound(16, 4) ** 2 - 0.2) <= 1e-16
    assert oracle.orthoplex_bound(16, 4) == 0.0       # needs N > d^2
    assert oracle.orthoplex_bound(17, 4) == 0.5
    # Levenshtein at N = d(d+1) equals 1/sqrt(d)
    for d in (2, 3, 4, 7):
        assert abs(oracle.levenshtein_bound(d * (d + 1), d) - 1 / math.sqrt(d)) <= 1e-15
    with pytest.raises(ValueError):
        oracle.welch_bound(1, 3)


@settings(max_examples=60, deadline=None)
@given(n=st.integers(2, 40), d=st.integers(1, 6), seed=st.integers(0, 2 ** 31))
def test_coherence_respects_lower_bounds(n, d, seed):
    F = inputs.random_frame(n, d, seed)
    mu = oracle.coherence(F)
    assert mu >= oracle.lower_bound(n, d) - 1e-12
    assert mu <= 1.0 + 1e-12


@settings(max_examples=30, deadline=None)
@given(n=st.integers(2, 24), d=st.integers(1, 6), seed=st.integers(0, 2 ** 31))
def test_invariances(n, d, seed):
    rng = np.random.default_rng(seed)
    F = inputs.random_frame(n, d, seed)
    mu = oracle.coherence(F)
    # left unitary
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)) + 1j * rng.standard_normal((d, d)))
    assert abs(oracle.coherence(Q @ F) - mu) <= 1e-13
    # per-column phases and positive scales
    ph = np.exp(2j * np.pi * rng.random(n)) * (0.1 + 10 * rng.random(n))
    assert abs(oracle.coherence(F * ph[None, :]) - mu) <= 1e-13
    # column permutation
    assert abs(oracle.coherence(F[:, rng.permutation(n)]) - mu) <= 1e-15
    # complex conjugation
    assert abs(oracle.coherence(np.conj(F)) - mu) <= 1e-15


def test_conjugation_matters_in_gram():
    """A Gram written without the conjugate (or transposed) gives other values
    on a complex frame; the coherence must come out as the SIC value."""
    F = frames.hesse_sic()
    wrong = np.abs(F.T @ F)
    np.fill_diagonal(wrong, 0)
    assert abs(wrong.max() - 0.5) > 1e-3
    assert abs(oracle.coherence(F) - 0.5) <= 1e-14


def test_zero_and_nonfinite_columns():
    F = inputs.random_frame(6, 3, 1)
    F[:, 2] = 0
    assert oracle.coherence(F) == math.inf
    F = inputs.random_frame(6, 3, 1)
    F[1, 4] = np.nan
    assert oracle.coherence(F) == math.inf
    _, norms = oracle.normalize_columns(inputs.random_frame(6, 3, 2))
    assert np.all(norms > 0)


def _pair_bruteforce(F):
    """Loops over j < k in order, keeping the first pair of largest squared
    modulus (inner products summed term by term)."""
    d, n = F.shape
    cols = [F[:, j] / math.sqrt(sum(abs(z) ** 2 for z in F[:, j])) for j in range(n)]
    best, bj, bk = -1.0, -1, -1
    for j in range(n):
        for k in range(j + 1, n):
            acc = 0j
            for i in range(d):
                acc += cols[j][i].conjugate() * cols[k][i]
            m = acc.real * acc.real + acc.imag * acc.imag
            if m > best:
                best, bj, bk = m, j, k
    return math.sqrt(best), bj, bk


@pytest.mark.parametrize("n,d,seed", [(2, 1, 0), (5, 3, 1), (9, 2, 2), (12, 4, 3), (7, 7, 4)])
def test_coherence_pair_bruteforce(n, d, seed):
    F = inputs.random_frame(n, d, seed=seed)
    mu, j, k = oracle.coherence_pair(F)
    mb, bj, bk = _pair_bruteforce(F)
    assert abs(mu - mb) <= 1e-13 and (j, k) == (bj, bk) and j < k
    assert abs(mu - oracle.coherence(F)) <= 1e-15


def test_coherence_pair_ties_and_invalid():
    """An orthonormal basis plus one repeated vector: the only nonzero pair
    is the repeat; e_1, e_2 and (e_1 + e_2) tie exactly at 1/sqrt 2 on the
    pairs (0, 2) and (1, 2), so the first, (0, 2), is returned; a zero
    column gives (inf, -1, -1)."""
    F = np.eye(4, dtype=complex)
    F = np.concatenate([F, F[:, 2:3] * 1j], axis=1)
    mu, j, k = oracle.coherence_pair(F)
    assert (j, k) == (2, 4) and abs(mu - 1.0) <= 1e-15
    mu, j, k = oracle.coherence_pair(np.array([[1.0, 0.0, 1.0], [0.0, 1.0, 1.0]], dtype=complex))
    assert (j, k) == (0, 2) and abs(mu - math.sqrt(0.5)) <= 2.3e-16   # the normalised entries are rounded
    F = inputs.random_frame(6, 3, seed=1)
    F[:, 3] = 0
    assert oracle.coherence_pair(F) == (math.inf, -1, -1)
