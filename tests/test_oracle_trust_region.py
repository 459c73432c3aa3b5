"""Pins of the oracle's trust-region step (Alg. 1 read with the textbook's
completion; outer ratio test) on quadratics with known answers."""

import math

import numpy as np
import pytest

import inputs
import oracle
from oracle.trust_region import (EXIT_BOUNDARY, EXIT_MAX_ITER, EXIT_NEGATIVE_CURVATURE, EXIT_SMALL_RESIDUAL,
                                 EXIT_ZERO_GRADIENT, fd_hess_vec)


def _quad(n, seed, shift=0.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.linspace(1.0, 10.0, n) + shift
    B = (Q * ev) @ Q.T
    g = rng.standard_normal(n)
    return B, g


def _model(B, g, p):
    return float(g @ p + 0.5 * p @ B @ p)


def test_interior_solution_is_newton_step():
    B, g = _quad(12, 0)
    p, it, code, Bp = oracle.cg_steihaug(g, lambda v: B @ v, 1e6, 1e-12, 50)
    assert code == EXIT_SMALL_RESIDUAL and it <= 13
    assert np.max(np.abs(p - np.linalg.solve(B, -g))) <= 1e-10
    assert np.max(np.abs(Bp - B @ p)) <= 1e-9


def test_boundary_step_length_and_cauchy_decrease():
    B, g = _quad(12, 1)
    for radius in (0.05, 0.2):
        p, it, code, Bp = oracle.cg_steihaug(g, lambda v: B @ v, radius, 1e-12, 50)
        assert code == EXIT_BOUNDARY
        assert abs(np.linalg.norm(p) - radius) <= 1e-12
        # at least the decrease of the Cauchy point (steepest descent to the boundary or model minimum)
        gBg = g @ B @ g
        tau = min(1.0, np.linalg.norm(g) ** 3 / (radius * gBg))
        pc = -tau * radius / np.linalg.norm(g) * g
        assert _model(B, g, p) <= _model(B, g, pc) + 1e-14
        assert np.max(np.abs(Bp - B @ p)) <= 1e-9


def test_negative_curvature_goes_to_the_better_boundary_point():
    B, g = _quad(8, 2, shift=-5.5)        # eigenvalues from -4.5 to 4.5
    rng = np.random.default_rng(3)
    for _ in range(5):
        g = rng.standard_normal(8)
        p, it, code, Bp = oracle.cg_steihaug(g, lambda v: B @ v, 0.3, 1e-12, 50)
        assert code in (EXIT_NEGATIVE_CURVATURE, EXIT_BOUNDARY)
        assert abs(np.linalg.norm(p) - 0.3) <= 1e-12
        assert np.max(np.abs(Bp - B @ p)) <= 1e-9
    # first direction already of negative curvature: -g with g an eigenvector of eigenvalue -2
    B = np.diag([-2.0, 1.0, 3.0])
    g = np.array([1.0, 0.0, 0.0])
    p, it, code, _ = oracle.cg_steihaug(g, lambda v: B @ v, 0.5, 1e-12, 10)
    assert code == EXIT_NEGATIVE_CURVATURE and it == 1
    assert np.allclose(p, [-0.5, 0.0, 0.0])          # the root with the lower model value, not +0.5


def test_zero_gradient_and_iteration_cap():
    B, g = _quad(6, 4)
    p, it, code, _ = oracle.cg_steihaug(np.zeros(6), lambda v: B @ v, 1.0, 1e-12, 10)
    assert code == EXIT_ZERO_GRADIENT and it == 0 and not np.any(p)
    p, it, code, _ = oracle.cg_steihaug(g, lambda v: B @ v, 1e6, 1e-30, 2)
    assert code == EXIT_MAX_ITER and it == 2


def test_fd_hessian_matches_second_differences_of_f():
    Y = inputs.random_frame(20, 3, seed=5)
    delta = 0.05
    rng = np.random.default_rng(6)
    hv = fd_hess_vec(Y, delta, 1e-6)
    for _ in range(3):
        v = rng.standard_normal(Y.shape) + 1j * rng.standard_normal(Y.shape)
        v /= math.sqrt(oracle.rdot(v, v))
        vbv = oracle.rdot(v, hv(v))
        h = 1e-4
        f = lambda X: oracle.smooth_max(X, delta)[1]
        second = (f(Y + h * v) - 2 * f(Y) + f(Y - h * v)) / (h * h)
        assert abs(vbv - second) <= 1e-4 * (1 + abs(vbv))


def test_tr_step_decreases_and_follows_the_radius_rules():
    Y = inputs.random_frame(40, 4, seed=1)
    p = oracle.TRParams(delta=0.05, radius=0.1)
    for _ in range(6):
        Y2, r = oracle.tr_step(Y, p)
        assert r.step_norm <= p.radius * (1 + 1e-12)
        if r.accepted:
            assert r.rho > p.eta and r.f_new < r.f_old
            assert np.array_equal(Y2, Y + (Y2 - Y))
        else:
            assert np.array_equal(Y2, Y)
        if r.rho < 0.25:
            assert r.new_radius == p.radius / 4
        elif r.rho > 0.75 and r.step_norm >= p.radius * (1 - 1e-12):
            assert r.new_radius == min(2 * p.radius, p.radius_max)
        else:
            assert r.new_radius == p.radius
        Y, p.radius = Y2, r.new_radius


def _table2():
    rows = {}
    import os
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "table2_trstmi_mu.txt")):
        if line.strip() and not line.startswith("#"):
            d, n, mu = line.split()
            rows[int(d)] = (int(n), float(mu))
    return rows


@pytest.mark.parametrize("d,restarts", [(2, 8), (3, 6), (4, 32), (5, 50)])
def test_optimize_reaches_table2(d, restarts):
    """Alg. 2 (continuation over delta, random restarts, trust-region steps)
    reaches the printed Table II coherence at N = d^2, which is also the
    Welch bound there, so the value is optimal."""
    n, printed = _table2()[d]
    mu, l, Y = oracle.optimize(n, d, oracle.OptParams(restarts=restarts))
    assert oracle.welch_bound(n, d) - 1e-12 <= mu <= printed
    assert abs(mu - oracle.coherence(Y)) == 0.0
