"""Pins of the oracle's smooth maximum (section IV: shifted log-sum-exp and
its Proposition), against closed forms, brute force and invariances."""

import math

import numpy as np
import pytest

import frames
import inputs
import oracle


@pytest.mark.parametrize("squared", [True, False])
@pytest.mark.parametrize("delta", [1.0, 0.1, 1e-2, 1e-4])
def test_proposition_bounds(delta, squared):
    # s <= F <= s + delta log n, n = N(N-1)/2 (the Proposition of section IV)
    for n_, d, seed in [(12, 3, 0), (40, 5, 1), (64, 8, 2)]:
        F = inputs.random_frame(n_, d, seed=seed)
        s, f = oracle.smooth_max(F, delta, squared)
        mu = oracle.coherence(F)
        assert abs(s - (mu * mu if squared else mu)) <= 1e-15
        n = n_ * (n_ - 1) // 2
        assert s <= f <= s + delta * math.log(n) * (1 + 1e-15)


@pytest.mark.parametrize("delta", [0.5, 0.05, 0.003])
def test_closed_form_three_vectors(delta):
    # e1, e2, (e1 + e2)/sqrt 2 in C^2: |G|^2 over j < k is {0, 1/2, 1/2}
    F = np.array([[1, 0, 1], [0, 1, 1]], dtype=complex)
    s, f = oracle.smooth_max(F, delta, squared=True)
    assert s == pytest.approx(0.5, abs=1e-15)
    assert f == pytest.approx(0.5 + delta * math.log(2 + math.exp(-0.5 / delta)), abs=1e-14)
    s, f = oracle.smooth_max(F, delta, squared=False)
    r = 1 / math.sqrt(2)
    assert s == pytest.approx(r, abs=1e-15)
    assert f == pytest.approx(r + delta * math.log(2 + math.exp(-r / delta)), abs=1e-14)


@pytest.mark.parametrize("name", ["three_lines", "tetrahedron", "simplex5", "hesse", "onb4"])
def test_equal_values_give_s_plus_delta_log_n(name):
    # every pair of an equiangular frame (or an orthonormal basis) has the same
    # |G|: F = s + delta log n exactly up to rounding
    build, mu = frames.KNOWN[name]
    F = build()
    n = F.shape[1] * (F.shape[1] - 1) // 2
    for delta in (0.1, 1e-3):
        s, f = oracle.smooth_max(F, delta)
        assert s == pytest.approx(mu * mu, abs=1e-14)
        assert f == pytest.approx(mu * mu + delta * math.log(n), abs=1e-12)


def test_numeric_sic_16_4():
    F = frames.sic_numeric(4)
    s, f = oracle.smooth_max(F, 0.01)
    assert abs(s - 0.2) <= 1e-13
    assert abs(f - (0.2 + 0.01 * math.log(120))) <= 1e-11


def test_monotone_in_delta_and_limits():
    F = inputs.random_frame(50, 6, seed=4)
    x = oracle.upper_values(F)
    vals = [oracle.smooth_max_of_values(x, dl)[1] for dl in (1e-6, 1e-4, 1e-2, 1.0)]
    assert all(a <= b for a, b in zip(vals, vals[1:]))   # dF/d delta = entropy >= 0
    s = float(np.max(x))
    assert abs(vals[0] - s) <= 1e-6 * math.log(len(x))    # delta -> 0: F -> s
    # delta -> infinity: F - delta log n -> mean(x), error about var(x) / (2 delta)
    dl = 1e4
    f = oracle.smooth_max_of_values(x, dl)[1]
    assert abs(f - dl * math.log(len(x)) - float(np.mean(x))) <= float(np.var(x)) / dl + 1e-9


def test_bruteforce_agrees():
    for n_, d, seed in [(5, 2, 0), (7, 3, 1), (9, 1, 2)]:
        F = inputs.random_frame(n_, d, seed=seed)
        for sq in (True, False):
            a = oracle.smooth_max(F, 0.05, sq)
            b = oracle.smooth_max_bruteforce(F, 0.05, sq)
            assert abs(a[0] - b[0]) <= 1e-15 and abs(a[1] - b[1]) <= 1e-14


def test_invariances():
    rng = np.random.default_rng(7)
    F = inputs.random_frame(30, 4, seed=7)
    s, f = oracle.smooth_max(F, 0.02)
    Q, _ = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
    phases = np.exp(2j * np.pi * rng.random(30))
    scales = rng.random(30) + 0.5
    G = (Q @ F)[:, rng.permutation(30)] * (phases * scales)[None, :]
    s2, f2 = oracle.smooth_max(G, 0.02)
    assert abs(s - s2) <= 1e-14 and abs(f - f2) <= 1e-13


def test_invalid_column_and_arguments():
    F = inputs.random_frame(10, 3, seed=0)
    F[:, 4] = 0
    assert oracle.smooth_max(F, 0.1) == (math.inf, math.inf)
    with pytest.raises(ValueError):
        oracle.smooth_max_of_values([0.1, 0.2], 0.0)


@pytest.mark.parametrize("n,d,delta", [(8, 2, 0.1), (20, 3, 0.05), (40, 6, 0.01)])
def test_gradient_matches_finite_differences(n, d, delta):
    rng = np.random.default_rng(n + d)
    Y = inputs.random_frame(n, d, seed=n) * (0.5 + rng.random(n))[None, :]
    g = oracle.smooth_max_grad(Y, delta)
    h = 1e-6
    for _ in range(4):
        E = rng.standard_normal(Y.shape) + 1j * rng.standard_normal(Y.shape)
        fd = (oracle.smooth_max(Y + h * E, delta)[1] - oracle.smooth_max(Y - h * E, delta)[1]) / (2 * h)
        an = float(np.sum((np.conj(g) * E).real))
        assert abs(fd - an) <= 1e-6 * (1 + abs(an))


def test_gradient_tangent_and_covariance():
    rng = np.random.default_rng(3)
    Y = inputs.random_frame(30, 4, seed=3)
    g = oracle.smooth_max_grad(Y, 0.02)
    Phi, norms = oracle.normalize_columns(Y)
    # F does not change when a column is scaled: no radial component
    assert np.max(np.abs(np.sum((Phi.conj() * g).real, axis=0))) <= 1e-13
    # column scales c_k and phases: g_k -> g_k e^{i t_k} / c_k
    c = 0.5 + rng.random(30)
    ph = np.exp(2j * np.pi * rng.random(30))
    g2 = oracle.smooth_max_grad(Y * (c * ph)[None, :], 0.02)
    assert np.max(np.abs(g2 - g * (ph / c)[None, :])) <= 1e-12
    # a unitary acting on the space: g -> Q g
    Q, _ = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
    g3 = oracle.smooth_max_grad(Q @ Y, 0.02)
    assert np.max(np.abs(g3 - Q @ g)) <= 1e-12
    Y[:, 2] = 0
    assert oracle.smooth_max_grad(Y, 0.02) is None
