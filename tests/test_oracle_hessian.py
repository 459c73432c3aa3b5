"""Pins of the oracle's exact Hessian-vector product of the smooth maximum
(B_k of Alg. 1 in section IV is the Hessian of the objective).

Each pin comes from outside the formula: a library's automatic
differentiation, the objective's invariances (column scale, column phase,
a common unitary map), the symmetry of a Hessian, second differences of the
objective itself, and the convergence order of central differences of the
gradient."""

import math

import numpy as np
import pytest

import inputs
import oracle
from oracle.smoothmax import smooth_max_hess_vec


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("n,d,delta", [(6, 2, 0.3), (9, 3, 0.05), (12, 4, 0.01)])
def test_matches_automatic_differentiation(n, d, delta):
    """torch's double backward of the objective (its own differentiation
    rules, nothing shared with the hand-derived chain) gives the same
    Hessian-vector product."""
    torch = pytest.importorskip("torch")
    Y = inputs.random_frame(n, d, seed=n)
    V = _rand(Y.shape, n + 1)

    def F(yr, yi):
        y = torch.complex(yr, yi)
        phi = y / torch.linalg.vector_norm(y, dim=0, keepdim=True)
        G = phi.conj().T @ phi
        iu = torch.triu_indices(n, n, offset=1)
        x = (G.real ** 2 + G.imag ** 2)[iu[0], iu[1]]
        s = x.max().detach()
        return s + delta * torch.log(torch.sum(torch.exp((x - s) / delta)))

    yr = torch.tensor(Y.real, dtype=torch.float64, requires_grad=True)
    yi = torch.tensor(Y.imag, dtype=torch.float64, requires_grad=True)
    vr = torch.tensor(V.real, dtype=torch.float64)
    vi = torch.tensor(V.imag, dtype=torch.float64)
    gr, gi = torch.autograd.grad(F(yr, yi), (yr, yi), create_graph=True)
    hr, hi = torch.autograd.grad((gr * vr).sum() + (gi * vi).sum(), (yr, yi))
    ref = hr.numpy() + 1j * hi.numpy()       # real-coordinate Hessian times V
    H = smooth_max_hess_vec(Y, V, delta)
    assert _rel(H, ref) <= 1e-11


def test_invariance_directions_have_closed_forms():
    """F is unchanged by y_k -> a y_k (a > 0), y_k -> e^{i t} y_k and Y -> U Y
    (U unitary), so along those curves the gradient is known exactly: the
    derivative of the gradient is -g_k, i g_k (column k only) and A g for
    U = exp(t A), A anti-Hermitian."""
    d, n, delta = 4, 14, 0.02
    Y = inputs.random_frame(n, d, seed=3) * np.linspace(0.5, 2.0, n)[None, :]
    g = oracle.smooth_max_grad(Y, delta)
    scale = 1e-12 * np.max(np.abs(g)) * 50
    for k in (0, 5, n - 1):
        V = np.zeros_like(Y)
        V[:, k] = Y[:, k]
        want = np.zeros_like(Y)
        want[:, k] = -g[:, k]
        assert np.max(np.abs(smooth_max_hess_vec(Y, V, delta) - want)) <= scale
        V[:, k] = 1j * Y[:, k]
        want[:, k] = 1j * g[:, k]
        assert np.max(np.abs(smooth_max_hess_vec(Y, V, delta) - want)) <= scale
    A = _rand((d, d), 4)
    A = A - A.conj().T
    assert np.max(np.abs(smooth_max_hess_vec(Y, A @ Y, delta) - A @ g)) <= scale * np.max(np.abs(A))


def test_symmetric_and_linear():
    d, n, delta = 3, 11, 0.05
    Y = inputs.random_frame(n, d, seed=8)
    U, V = _rand(Y.shape, 9), _rand(Y.shape, 10)
    HU, HV = smooth_max_hess_vec(Y, U, delta), smooth_max_hess_vec(Y, V, delta)
    a, b = oracle.rdot(U, HV), oracle.rdot(V, HU)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
    HW = smooth_max_hess_vec(Y, 2.5 * U - 0.75 * V, delta)
    assert _rel(HW, 2.5 * HU - 0.75 * HV) <= 1e-13


def test_curvature_equals_second_differences_of_f():
    """<v, H v> is the second derivative of F along v: a fourth-order
    five-point stencil of F values agrees to its truncation error."""
    Y = inputs.random_frame(20, 3, seed=5)
    delta = 0.05
    f = lambda X: oracle.smooth_max(X, delta)[1]
    for seed in range(3):
        v = _rand(Y.shape, 20 + seed)
        v /= math.sqrt(oracle.rdot(v, v))
        vhv = oracle.rdot(v, smooth_max_hess_vec(Y, v, delta))
        h = 2e-3
        second = (-f(Y + 2 * h * v) + 16 * f(Y + h * v) - 30 * f(Y) + 16 * f(Y - h * v) - f(Y - 2 * h * v)) / (12 * h * h)
        assert abs(vhv - second) <= 1e-6 * (1 + abs(vhv))


def test_central_differences_of_the_gradient_converge_at_second_order():
    """The central difference of the gradient differs from the exact product
    by c h^2 + O(h^4): dividing h by 10 divides the difference by about 100,
    which a wrong exact product would not allow."""
    Y = inputs.random_frame(16, 4, seed=12)
    V = _rand(Y.shape, 13)
    delta = 0.03
    H = smooth_max_hess_vec(Y, V, delta)
    errs = []
    for h in (1e-4, 1e-5):
        fd = (oracle.smooth_max_grad(Y + h * V, delta) - oracle.smooth_max_grad(Y - h * V, delta)) / (2 * h)
        errs.append(np.max(np.abs(fd - H)))
    assert 80.0 <= errs[0] / errs[1] <= 120.0
    assert errs[1] <= 1e-6 * np.max(np.abs(H))


def test_invalid_column_gives_none():
    Y = inputs.random_frame(8, 3, seed=1)
    Y[:, 2] = 0.0
    assert smooth_max_hess_vec(Y, _rand(Y.shape, 2), 0.1) is None
