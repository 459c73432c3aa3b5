"""Trust-region step of the paper's optimiser (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Alg. 1 of the paper is Steihaug's truncated conjugate gradient for the
trust-region subproblem (its dagger): minimise m(p) = f + g.p + p.B p / 2
subject to |p| <= radius, B the Hessian of f.  The printed listing is
garbled; it is read with the textbook's completion (Nocedal & Wright,
Alg. 7.2, which the paper cites): the boundary test is on the new iterate
z_{j+1}, the residual test on the new residual r_{j+1}, and the missing
update beta = r_{j+1}.r_{j+1} / r_j.r_j, d_{j+1} = -r_{j+1} + beta d_j is
added.  With negative curvature the step goes to the boundary point on the
line z_j + tau d_j with the lower model value.

The outer step is the textbook trust-region iteration (Nocedal & Wright,
Alg. 4.1): rho = (f(Y) - f(Y + p)) / (m(0) - m(p)); rho < 1/4 shrinks the
radius by 4; rho > 3/4 with the step on the boundary doubles it (up to a
maximum); the step is taken when rho > eta.  Hessian-vector products are
exact (B = the Hessian of the objective, as Alg. 1's dagger states:
``smooth_max_hess_vec``); central differences of the gradient along the
unit direction remain as an option (``fd_step > 0``).

Vectors are the real coordinates of a complex d x N frame: the dot product
is sum Re(conj(u) v) and the gradient is ``smooth_max_grad``.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .smoothmax import smooth_max, smooth_max_grad, smooth_max_hess_vec

EXIT_SMALL_RESIDUAL = 0
EXIT_NEGATIVE_CURVATURE = 1
EXIT_BOUNDARY = 2
EXIT_MAX_ITER = 3
EXIT_ZERO_GRADIENT = 4


def rdot(u, v):
    """sum Re(conj(u) v): the real inner product of the frame coordinates."""
    return float(np.sum((np.conj(u) * v).real))


def _to_boundary(z, d, radius):
    """The two tau with |z + tau d| = radius (tau_minus <= 0 <= tau_plus
    when |z| <= radius)."""
    a = rdot(d, d)
    b = 2.0 * rdot(z, d)
    c = rdot(z, z) - radius * radius
    disc = math.sqrt(max(b * b - 4.0 * a * c, 0.0))
    return (-b - disc) / (2.0 * a), (-b + disc) / (2.0 * a)


def cg_steihaug(g, hess_vec, radius, tol, max_iter):
    """Steihaug CG for min g.p + p.B p / 2, |p| <= radius (Alg. 1, read as
    above).  Returns (p, iterations, exit code, B p)."""
    z = np.zeros_like(g)
    Bz = np.zeros_like(g)
    r = g.copy()
    d = -r
    rr = rdot(r, r)
    if math.sqrt(rr) < tol:
        return z, 0, EXIT_ZERO_GRADIENT, Bz
    for j in range(max_iter):
        Bd = hess_vec(d)
        dBd = rdot(d, Bd)
        if dBd <= 0.0:
            tm, tp = _to_boundary(z, d, radius)

            def model(t):  # g.p + p.B p / 2 along p = z + t d
                return (rdot(g, z) + t * rdot(g, d) + 0.5 * (rdot(z, Bz) + 2 * t * rdot(d, Bz) + t * t * dBd))

            t = tm if model(tm) < model(tp) else tp
            return z + t * d, j + 1, EXIT_NEGATIVE_CURVATURE, Bz + t * Bd
        alpha = rr / dBd
        z_new = z + alpha * d
        if math.sqrt(rdot(z_new, z_new)) >= radius:
            _, tp = _to_boundary(z, d, radius)
            return z + tp * d, j + 1, EXIT_BOUNDARY, Bz + tp * Bd
        r_new = r + alpha * Bd
        Bz = Bz + alpha * Bd
        rr_new = rdot(r_new, r_new)
        if math.sqrt(rr_new) < tol:
            return z_new, j + 1, EXIT_SMALL_RESIDUAL, Bz
        beta = rr_new / rr
        d = -r_new + beta * d
        z, r, rr = z_new, r_new, rr_new
    return z, max_iter, EXIT_MAX_ITER, Bz


@dataclass
class TRParams:
    delta: float = 1e-2          # smoothing of the maximum
    radius: float = 0.1
    radius_max: float = 1.0
    eta: float = 0.1
    cg_tol: float = 1e-8
    cg_max_iter: int = 20
    fd_step: float = 0.0         # 0: exact Hessian products; > 0: central differences with this step


@dataclass
class TRReport:
    f_old: float
    f_new: float
    rho: float
    step_norm: float
    new_radius: float
    cg_iters: int
    cg_exit: int
    accepted: bool


def fd_hess_vec(Y, delta, h):
    """v -> B v by central differences of the gradient along v / |v|."""
    def hv(v):
        nv = math.sqrt(rdot(v, v))
        if nv == 0.0:
            return np.zeros_like(v)
        u = v / nv
        gp = smooth_max_grad(Y + h * u, delta)
        gm = smooth_max_grad(Y - h * u, delta)
        return (gp - gm) * (nv / (2.0 * h))
    return hv


def exact_hess_vec(Y, delta):
    """v -> B v with B the exact Hessian of the smooth maximum at Y."""
    def hv(v):
        return smooth_max_hess_vec(Y, v, delta)
    return hv


def tr_step(Y, p: TRParams):
    """One outer trust-region iteration on the smooth maximum over |G|^2.
    Returns (new frame, report)."""
    Y = np.asarray(Y, dtype=np.complex128)
    f0 = smooth_max(Y, p.delta)[1]
    g = smooth_max_grad(Y, p.delta)
    hv = fd_hess_vec(Y, p.delta, p.fd_step) if p.fd_step > 0 else exact_hess_vec(Y, p.delta)
    step, iters, code, Bstep = cg_steihaug(g, hv, p.radius, p.cg_tol, p.cg_max_iter)
    snorm = math.sqrt(rdot(step, step))
    pred = -(rdot(g, step) + 0.5 * rdot(step, Bstep))
    if snorm == 0.0 or not pred > 0.0:
        return Y.copy(), TRReport(f0, f0, 0.0, snorm, p.radius / 4, iters, code, False)
    f1 = smooth_max(Y + step, p.delta)[1]
    rho = (f0 - f1) / pred
    radius = p.radius
    if rho < 0.25:
        radius = p.radius / 4
    elif rho > 0.75 and snorm >= p.radius * (1 - 1e-12):
        radius = min(2 * p.radius, p.radius_max)
    accepted = rho > p.eta
    return (Y + step if accepted else Y.copy()), TRReport(f0, f1, rho, snorm, radius, iters, code, accepted)


@dataclass
class OptParams:
    restarts: int = 8                     # L random starts (the paper uses L = 2 d^2)
    deltas: tuple = (1e-1, 3e-2, 1e-2, 3e-3, 1e-3, 3e-4, 1e-4)   # decreasing smoothing (continuation)
    steps_per_delta: int = 40
    radius0: float = 0.1                  # radius at the start of every delta
    radius_min: float = 1e-10             # a delta ends when the radius falls below this
    radius_max: float = 1.0
    eta: float = 0.1
    cg_tol: float = 1e-10
    cg_max_iter: int = 0                  # 0: 2 d N (the dimension of the real search space)
    fd_step: float = 0.0                  # 0: exact Hessian products
    seed: int = 0


def optimize(n, d, op: OptParams):
    """The paper's outer procedure (Alg. 2): for each of L random starts
    (the Haar start of stream l), minimise F_{s,delta_k} with trust-region
    steps for a decreasing sequence of delta_k, feeding each minimiser to the
    next; keep the frame with the smallest coherence.  Returns
    (best mu, best restart index, best frame)."""
    from .trstmi import Params, haar_init
    from .coherence import coherence

    best = (math.inf, -1, None)
    for l in range(op.restarts):
        Y = haar_init(Params(n=n, d=d, seed=op.seed, stream_id=l)).frame
        for dl in op.deltas:
            p = TRParams(delta=dl, radius=op.radius0, radius_max=op.radius_max, eta=op.eta, cg_tol=op.cg_tol,
                         cg_max_iter=op.cg_max_iter or 2 * d * n, fd_step=op.fd_step)
            for _ in range(op.steps_per_delta):
                Y, r = tr_step(Y, p)
                p.radius = r.new_radius
                if p.radius < op.radius_min or r.cg_exit == EXIT_ZERO_GRADIENT:
                    break
        mu = coherence(Y)
        if mu < best[0]:
            best = (mu, l, Y)
    return best
