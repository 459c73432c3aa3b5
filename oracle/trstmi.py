"""Stochastic trust-region candidate search on the coherence (oracle, FP64).

What the paper fixes: the objective is the coherence of the column-normalised
frame (§I; §IV on normalising each column and on using the upper triangle of
|Gram|), the search starts from a random collection of unit vectors (Alg. 2
step 1), and the search is a trust-region method over a radius (Alg. 1).

What the paper leaves open and this project reads as follows (each reading is
listed with its reason in the design notes):

* a step draws C candidates  Y_c = Phi_t + (Delta_t / sqrt(d)) Z_{t,c},
  Z i.i.d. CN(0, 1) (``rng``), so each column moves by Delta_t in RMS norm;
* every candidate is renormalised column by column; a column of norm zero or
  a non-finite norm makes the candidate invalid (its coherence is +inf);
* mu_c = coherence(Phi_c); the best candidate is c* = argmin over (mu_c, c),
  so ties go to the lowest index;
* accept iff mu_{c*} < mu_t (strict); on accept the frame becomes Phi_{c*}
  and the radius grows, Delta <- min(grow * Delta, Delta_max); otherwise the
  frame stays and the radius shrinks, Delta <- max(shrink * Delta, Delta_min);
* stop when mu_t <= target (if a target is set) or t = max_steps.

Reduced-precision forms (emulated here in FP64 arithmetic on rounded inputs):

* ``fp32``: candidates are rounded to binary32 before the Gram; mu_c is the
  coherence of the rounded candidate;
* ``bf16``: every candidate is screened with its entries rounded to
  bfloat16; the ``recheck_topk`` candidates with the smallest screened value
  (ties to the lowest index) are evaluated exactly in FP64, and select/accept
  use those FP64 values only.
"""

from __future__ import annotations

import dataclasses
import functools
import math
from typing import Optional

import numpy as np

from .coherence import normalize_columns
from .rng import TAG_HAAR, TAG_PERTURB, complex_gaussian_frame
from .rounding import round_complex, round_to_bf16, round_to_fp32

MODES = ("fp64", "fp32", "bf16")

# Default near-tie thresholds: a decision that depends on two values closer
# than this is reported as a near tie (decisions may then differ between two
# correct implementations that round differently).
NEAR_TIE = {"fp64": 2e-12, "fp32": 4e-6, "bf16": 2e-12}
SCREEN_NEAR_TIE = 2e-5


@dataclasses.dataclass
class Params:
    n: int
    d: int
    candidates: int = 64
    mode: str = "fp64"
    recheck_topk: int = 8
    seed: int = 0
    stream_id: int = 0
    radius0: float = 0.1
    grow: float = 2.0
    shrink: float = 0.5
    radius_min: float = 1e-12
    radius_max: float = 1.0
    max_steps: int = 1000
    target_mu: float = 0.0
    near_tie: Optional[float] = None

    def tie_threshold(self):
        return NEAR_TIE[self.mode] if self.near_tie is None else self.near_tie


@dataclasses.dataclass
class State:
    frame: np.ndarray          # (d, n) complex128, unit columns
    mu: float
    radius: float
    t: int = 0
    done: bool = False

    def copy(self):
        return State(self.frame.copy(), self.mu, self.radius, self.t, self.done)


@dataclasses.dataclass
class StepReport:
    cand_mu: np.ndarray         # (C,) mu_c as the mode computes it (screened value in bf16 mode)
    cand_mu_fp64: np.ndarray    # (C,) exact FP64 coherence of every candidate
    valid: np.ndarray           # (C,) bool
    rechecked: Optional[np.ndarray]   # bf16 mode: candidate indices evaluated in FP64, by screened rank
    best: int                   # c*, -1 if no valid candidate
    best_mu: float              # the value the accept test used for c*
    accepted: bool
    near_tie: bool
    screen_gap: float           # bf16 mode: gap between the k-th and (k+1)-th screened values


@functools.lru_cache(maxsize=16)
def _upper_mask(n):
    return np.triu(np.ones((n, n), dtype=bool), k=1)


def _max_sq_offdiag(Phi):
    """max_{j<k} |<phi_j, phi_k>|^2 for a frame with unit columns (FP64 Gram)."""
    G = Phi.conj().T @ Phi
    a = G.real * G.real + G.imag * G.imag
    return float(np.max(a[_upper_mask(Phi.shape[1])]))


def haar_init(p: Params) -> State:
    """Random start (Alg. 2 step 1): columns are normalised CN(0, I_d) vectors,
    drawn with tag 1, candidate 0, step 0.  The start's coherence is exact FP64
    in every mode (the FP32 mode reports it as the binary32 path computes it)."""
    Z = complex_gaussian_frame(p.n, p.d, p.seed, p.stream_id, 0, 0, TAG_HAAR)
    Phi, norms = normalize_columns(Z)
    if not np.all(np.isfinite(norms) & (norms > 0)):
        raise FloatingPointError("random start produced a zero column")
    mu = math.sqrt(_max_sq_offdiag(_rounded(Phi, "fp32" if p.mode == "fp32" else "fp64")))
    return State(frame=Phi, mu=mu, radius=float(p.radius0), t=0, done=_is_done(p, mu, 0))


def perturbations(p: Params, t: int, cands=None):
    """Z_{t,c} for the given candidates (all C by default): shape (C, d, n)."""
    if cands is None:
        cands = np.arange(p.candidates)
    return complex_gaussian_frame(p.n, p.d, p.seed, p.stream_id, np.asarray(cands), t, TAG_PERTURB)


def make_candidates(frame, radius, d, Z):
    """Y_c = Phi + (Delta / sqrt(d)) Z_c, then column normalisation.

    Returns (Phi_c of shape (C, d, n), valid of shape (C,)).
    """
    s = radius / math.sqrt(d)
    C = Z.shape[0]
    out = np.empty_like(Z)
    valid = np.ones(C, dtype=bool)
    for c in range(C):
        Phi, norms = normalize_columns(frame + s * Z[c])
        valid[c] = bool(np.all(np.isfinite(norms) & (norms > 0)))
        out[c] = Phi
    return out, valid


def _rounded(Phi, mode):
    if mode == "fp32":
        return round_complex(Phi, round_to_fp32)
    if mode == "bf16":
        return round_complex(Phi, round_to_bf16)
    return Phi


def evaluate_candidates(Phi_c, valid, mode="fp64"):
    """mu_c of each candidate computed on its entries rounded for ``mode``
    (``fp64``: unrounded).  Invalid candidates get +inf."""
    C = Phi_c.shape[0]
    mu = np.full(C, math.inf)
    for c in range(C):
        if valid[c]:
            mu[c] = math.sqrt(_max_sq_offdiag(_rounded(Phi_c[c], mode)))
    return mu


def _argmin_lowest(values, allowed=None):
    """Index of the smallest value, ties to the lowest index; -1 if none is finite."""
    best, best_v = -1, math.inf
    for c, v in enumerate(values):
        if allowed is not None and not allowed[c]:
            continue
        if v < best_v:
            best, best_v = c, v
    return best


def screen_error_bound(d):
    """Largest possible |screened - exact| coherence for unit columns in C^d.

    Input rounding: rounding the real and imaginary parts of an entry to
    bfloat16 (relative error at most u = 2^-8 each) moves the complex entry by
    at most u times its modulus, so a unit column moves by at most u in norm
    and, by the triangle and Cauchy-Schwarz inequalities, the complex inner
    product of two unit columns moves by at most 2u + u^2.

    Accumulation: products of two bfloat16 values are exact in binary32; Re
    and Im are each a sum of 2d such products, whose absolute values add up to
    at most |phi^| |psi^| <= (1 + u)^2.  Assuming only that every addition of
    the binary32 accumulation is faithful (its error is below one ulp of its
    result, in whatever direction the hardware rounds or truncates), each sum
    is off by at most gamma_{2d} (1 + u)^2 with gamma_n = n w / (1 - n w),
    w = 2^-23 (round to nearest alone would allow 2^-24); Re and Im together
    give the factor sqrt(2).

    Epilogue: a few binary32 roundings in |G|^2 and the square root (8 v,
    v = 2^-24), and the FP64 value's own rounding (1e-12).
    """
    u = 2.0 ** -8
    w = 2.0 ** -23
    v = 2.0 ** -24
    n = 2 * d
    gamma = n * w / (1.0 - n * w)
    return (2 * u + u * u) + math.sqrt(2.0) * gamma * (1 + u) ** 2 + 8 * v + 1e-12


def split_screen_error_bound(d):
    """Largest possible |screened - exact| coherence for unit columns in C^d
    under the batched form's split screen.

    Input: each real component x of a unit column is rounded to binary32
    (f, relative error at most 2^-24) and held as hi + lo, hi the bfloat16
    rounding of f and lo the bfloat16 rounding of the exact remainder
    r = f - hi.  With 2^e <= |f| < 2^(e+1), |r| is at most half the bfloat16
    spacing of that binade, 2^(e-8); at equality r is a power of two and lo =
    r; otherwise |r| < 2^(e-8), so r lies in a binade at or below 2^(e-9) and
    |lo - r| <= 2^(e-9-8) <= 2^-17 |f|.  hi + lo is therefore within delta =
    2^-17 (1 + 2^-24) + 2^-24 of x, relative; a complex entry moves by at
    most delta times its modulus and the inner product of two unit columns by
    at most 2 delta + delta^2.

    Products: Re and Im are each formed from the three products
    hi hi' + hi lo' + lo hi' of every real pair (each exact in binary32);
    |r| <= u |f| and |lo| <= (1 + u) |r| with u = 2^-8, so the dropped lo lo'
    add up to at most 2^-16 (1 + u)^2 (1 + 2^-24)^2.

    Accumulation: 3 x 32 products per part (the K = 2d <= 32 reals padded with
    zeros), every binary32 addition faithful (error below one ulp, w =
    2^-23): gamma_96 times the sum of |products|, which is at most
    (1 + u)^2 (1 + 2u) (1 + 2^-24)^2.  Re and Im together give the factor
    sqrt(2) on the product and accumulation terms.

    Epilogue: the binary32 |G|^2 and the FP64 square root and threshold
    (16 v, v = 2^-24), and the FP64 value's own rounding (1e-12).
    """
    if d > 16:
        raise ValueError("the split screen serves d <= 16 (one 32-real MFMA step)")
    u = 2.0 ** -8
    v = 2.0 ** -24
    w = 2.0 ** -23
    delta = 2.0 ** -17 * (1 + v) + v
    inputs = 2 * delta + delta * delta
    unit = (1 + v) ** 2
    dropped = 2.0 ** -16 * (1 + u) ** 2 * unit
    n = 96
    gamma = n * w / (1.0 - n * w)
    accumulation = gamma * (1 + u) ** 2 * (1 + 2 * u) * unit
    return inputs + math.sqrt(2.0) * (dropped + accumulation) + 16 * v + 1e-12


def _is_done(p, mu, t):
    return (p.target_mu > 0 and mu <= p.target_mu) or t >= p.max_steps


def step(p: Params, state: State, Z=None, exact_all=True):
    """One step of the candidate search from ``state`` (not modified).

    ``Z`` (shape (C, d, n)) replaces the generator's draws when given.
    ``exact_all=False`` (bf16 mode only) evaluates the exact FP64 coherence
    of the rechecked candidates only, the only ones any decision reads; the
    others get NaN in ``cand_mu_fp64``.
    Returns (new_state, StepReport).
    """
    if p.mode not in MODES:
        raise ValueError(p.mode)
    if state.done:
        return state.copy(), None
    C = p.candidates
    if Z is None:
        Z = perturbations(p, state.t)
    Phi_c, valid = make_candidates(state.frame, state.radius, p.d, Z)
    skip = p.mode == "bf16" and not exact_all
    mu64 = np.full(C, math.nan) if skip else evaluate_candidates(Phi_c, valid, "fp64")
    tau = p.tie_threshold()
    rechecked = None
    screen_gap = math.inf
    if p.mode == "fp64":
        cand_mu = mu64
        used = mu64
        best = _argmin_lowest(used)
    elif p.mode == "fp32":
        cand_mu = evaluate_candidates(Phi_c, valid, "fp32")
        used = cand_mu
        best = _argmin_lowest(used)
    else:
        cand_mu = evaluate_candidates(Phi_c, valid, "bf16")
        k = min(p.recheck_topk, C)
        order = sorted(range(C), key=lambda c: (cand_mu[c], c))
        rechecked = np.array(order[:k], dtype=np.int64)
        if skip:
            mu64[rechecked] = evaluate_candidates(Phi_c[rechecked], valid[rechecked], "fp64")
        if k < C:
            screen_gap = float(cand_mu[order[k]] - cand_mu[order[k - 1]])
        allowed = np.zeros(C, dtype=bool)
        allowed[rechecked] = True
        used = mu64
        best = _argmin_lowest(used, allowed)

    best_mu = float(used[best]) if best >= 0 else math.inf
    accepted = best >= 0 and best_mu < state.mu
    # near ties: the accept test, or the choice between the two best candidates
    cands_for_tie = used if rechecked is None else used[rechecked]
    finite = np.sort(cands_for_tie[np.isfinite(cands_for_tie)])
    near = best >= 0 and abs(best_mu - state.mu) <= tau
    if finite.size >= 2 and finite[1] - finite[0] <= tau:
        near = True
    if rechecked is not None and screen_gap <= SCREEN_NEAR_TIE:
        near = True

    new = state.copy()
    if accepted:
        new.frame = Phi_c[best].copy()
        new.mu = best_mu
        new.radius = min(state.radius * p.grow, p.radius_max)
    else:
        new.radius = max(state.radius * p.shrink, p.radius_min)
    new.t = state.t + 1
    new.done = _is_done(p, new.mu, new.t)
    rep = StepReport(cand_mu=cand_mu, cand_mu_fp64=mu64, valid=valid, rechecked=rechecked,
                     best=best, best_mu=best_mu, accepted=accepted, near_tie=near,
                     screen_gap=screen_gap)
    return new, rep


def solve(p: Params, state: Optional[State] = None, record=False):
    """Run steps until done.  Returns (final_state, history) where history is a
    list of (t, mu, radius, accepted, near_tie) per step when ``record``."""
    st = haar_init(p) if state is None else state.copy()
    hist = []
    while not st.done:
        st, rep = step(p, st)
        if record:
            hist.append((st.t, st.mu, st.radius, rep.accepted, rep.near_tie))
    return st, hist
