"""Pins of the BF16 screen's certified error bound (``oracle.screen_error_bound``).

The precision form screens every candidate from bfloat16 inputs with binary32
accumulation and trusts the screened values only to within the bound: the
tiles and candidates it prunes are provably below the exact FP64 maximum only
if |screened - exact| never exceeds it.  These tests pin the bound against
adversarial inputs rather than against random frames, where the error is an
order of magnitude below it:

* input rounding: unit columns whose real components all sit just beside a
  bfloat16 midpoint, on the side that makes every rounding error push the
  inner product the same way, reach almost the whole input term 2u + u^2 --
  and so exceed a bound that counts the rounding of only one column;
* accumulation: a binary32 sum whose additions truncate (a faithful but not
  round-to-nearest accumulation, which the bound allows for) exceeds the
  round-to-nearest form of the summation lemma (unit roundoff 2^-24) and stays
  within the form the bound uses (2^-23); a bound without an accumulation
  term is exceeded by it;
* both together on a frame, and random frames under every rounding direction
  of the accumulation, stay within the bound.

The accumulation emulation below is a test helper: the oracle's own bf16 form
evaluates the Gram of the rounded inputs in FP64 (no accumulation error).
"""

import math

import numpy as np
import pytest

import oracle

U = 2.0 ** -8          # bfloat16 unit roundoff (round to nearest even)
W = 2.0 ** -23         # faithful binary32 addition: error below one ulp


def _bf16_ulp(x):
    """Spacing of bfloat16 values around |x| (normal range)."""
    _, e = math.frexp(abs(x))          # |x| = m 2^e, 1/2 <= m < 1
    return 2.0 ** (e - 8)


def _frac_in_ulp(x):
    """Position of |x| between the two bfloat16 values around it, in [0, 1)."""
    q = _bf16_ulp(x)
    return abs(x) / q - math.floor(abs(x) / q)


def _rounds_up(x):
    """True when round-to-nearest-even to bfloat16 increases |x|."""
    return abs(float(oracle.round_to_bf16(np.array([x]))[0])) > abs(x)


def adversarial_pair(d, c_range=(0.3, 0.7), seed=0):
    """Two unit columns phi, psi in C^d (d >= 4) with equal component moduli
    and <phi, psi> = c real in ``c_range``, built so that rounding to
    bfloat16 raises Re<phi, psi> by about 2u.

    The relative error of rounding x to bfloat16 is about u only when x sits
    next to a midpoint whose mantissa is close to 1, so m = min(2d, 16) - 2
    real components (the first m/2 complex entries) are drawn from the
    midpoints (1 + k 2^-8) 2^e, k in {1, 3, 5, 7, 9}, moved by a relative 1e-5
    off the midpoint:

    * "agree" components carry the same sign in phi and psi and sit just above
      their midpoint (round up);
    * "disagree" components carry opposite signs and sit just below it
      (round down).

    One more component t = sqrt(1 - sum of their squares) makes the norm 1
    (t^2 <= 0.02 is kept small: its rounding is not chosen) and joins the
    group its own rounding direction calls for; the partner of t and every
    other entry are zero, which rounds exactly.  Then
    Re<phi^, psi^> = sum_agree x^2 (1 + u_i)^2 - sum_disagree x^2 (1 - u_i)^2
    = c + 2 sum_i u_i x_i^2 ~ c + 2u.  The real and imaginary parts of one
    complex entry share their group, so Im<phi, psi> = 0 before and after
    rounding.
    """
    assert d >= 4
    rng = np.random.default_rng(seed)
    mids = np.array([(1 + k * 2.0 ** -8) * 2.0 ** e for k in (1, 3, 5, 7, 9) for e in range(-1, -8, -1)])
    m = min(2 * d, 16) - 2                                         # midpoint components
    for n_up in (m // 2 + 1 - (m // 2 + 1) % 2, m // 2 - 1 + (m // 2 + 1) % 2):
        sign = np.array([1.0] * n_up + [-1.0] * (m - n_up))     # +1: agree, rounds up
        idx = rng.integers(0, mids.size, size=(400000, m))
        x0 = mids[idx] * (1 + 1e-5 * sign)
        sq = x0 * x0
        total = sq.sum(axis=1)
        c0 = (sq * sign).sum(axis=1)
        ok = (total < 1.0) & (total >= 0.98) & (c0 >= c_range[0] + 0.02) & (c0 <= c_range[1] - 0.02)
        if not ok.any():
            continue
        x = x0[int(np.flatnonzero(ok)[0])]
        t = math.sqrt(1.0 - math.fsum((x * x).tolist()))
        comps = np.zeros(2 * d)
        comps[:m] = x
        comps[m] = t                                              # comps[m + 1] (its partner) stays 0
        signs = np.ones(2 * d)
        signs[n_up:m] = -1.0
        signs[m] = 1.0 if _rounds_up(t) else -1.0
        phi = comps[0::2] + 1j * comps[1::2]
        psi = (comps * signs)[0::2] + 1j * (comps * signs)[1::2]
        # unit up to FP64 rounding; normalised the way the path does (FP64)
        phi, psi = phi / np.linalg.norm(phi), psi / np.linalg.norm(psi)
        for v, sg in zip(comps[:m], sign):
            assert _rounds_up(v) == (sg > 0)                      # every component rounds its group's way
        return phi, psi
    raise AssertionError("no adversarial construction found")


def _rounded(z):
    return oracle.round_to_bf16(z.real) + 1j * oracle.round_to_bf16(z.imag)


def fp32_sum(terms, direction):
    """Sequential binary32 sum of exactly representable terms; each addition
    rounds the exact (FP64) sum to binary32 in ``direction``: 'nearest',
    'zero' (truncation), 'up' or 'down'."""
    acc = np.float32(0.0)
    for t in terms:
        exact = float(acc) + float(t)
        r = np.float32(exact)
        if direction == "zero" and abs(float(r)) > abs(exact):
            r = np.nextafter(r, np.float32(0.0))
        elif direction == "up" and float(r) < exact:
            r = np.nextafter(r, np.float32(np.inf))
        elif direction == "down" and float(r) > exact:
            r = np.nextafter(r, np.float32(-np.inf))
        acc = r
    return float(acc)


def screened_inner(phi_r, psi_r, direction):
    """<phi^, psi^> of bf16-valued columns with each real part accumulated as
    a binary32 sum of its 2d exact products in ``direction``."""
    re_terms = np.concatenate([phi_r.real * psi_r.real, phi_r.imag * psi_r.imag])
    im_terms = np.concatenate([phi_r.real * psi_r.imag, -(phi_r.imag * psi_r.real)])
    return complex(fp32_sum(re_terms, direction), fp32_sum(im_terms, direction))


@pytest.mark.parametrize("d", [4, 16, 64, 128])
def test_input_rounding_reaches_the_input_term(d):
    phi, psi = adversarial_pair(d)
    F = np.stack([phi, psi], axis=1)
    exact = oracle.coherence(F)
    # the oracle's own bf16 form: entries rounded, Gram of the rounded values in FP64
    screen = float(oracle.evaluate_candidates(F[None], np.array([True]), "bf16")[0])
    err = screen - exact
    eps = oracle.screen_error_bound(d)
    assert 0.3 <= exact <= 0.7
    assert err <= eps
    # nearly the whole input term is attained ...
    assert err >= 0.93 * (2 * U + U * U)
    # ... so a bound that counted the rounding of one column only is exceeded
    one_column = (U + U * U) + (eps - (2 * U + U * U))
    assert err > one_column


def test_input_rounding_direct_inner_product():
    """The same construction read directly: Re<phi^, psi^> - <phi, psi> ~ 2u
    and the imaginary part stays zero."""
    phi, psi = adversarial_pair(64)
    g = np.vdot(phi, psi)
    gr = np.vdot(_rounded(phi), _rounded(psi))
    assert abs(g.imag) <= 1e-15 and abs(gr.imag) <= 1e-15
    assert 0.93 * 2 * U <= gr.real - g.real <= 2 * U + U * U


def test_truncating_accumulation_exceeds_the_round_to_nearest_lemma():
    """Sum of 2d = 128 exact bf16 products: 0.75^2, then 127 products just
    below one binary32 ulp of the partial sum (2^-24 (1 - 2^-8)^2).  Truncating
    additions drop every one of them.  The error exceeds gamma_n(2^-24) times
    the sum of |terms| and stays within gamma_n(2^-23) times it."""
    n = 128
    a = np.array([0.75] + [2.0 ** -12 * (1 - 2.0 ** -8)] * (n - 1))
    assert np.array_equal(oracle.round_to_bf16(a), a)       # exact bf16 inputs
    terms = a * a                                           # exact products
    exact = math.fsum(terms.tolist())
    trunc = fp32_sum(terms, "zero")
    assert trunc == 0.75 ** 2                               # every small term lost
    err = exact - trunc
    s_abs = math.fsum(np.abs(terms).tolist())
    gamma24 = n * 2.0 ** -24 / (1 - n * 2.0 ** -24)
    gamma23 = n * W / (1 - n * W)
    assert err > gamma24 * s_abs
    assert err <= gamma23 * s_abs
    # round to nearest keeps them (each is above half an ulp), within the 2^-24 lemma
    assert abs(exact - fp32_sum(terms, "nearest")) <= gamma24 * s_abs


def test_bound_without_accumulation_term_is_exceeded():
    """Exactly representable unit-norm inputs (no input rounding at all): the
    truncating accumulation alone exceeds a bound made of the input and
    epilogue terms only, and stays within the full bound."""
    d = 64
    # unit column of bf16 values: 0.75 e_1 plus 127 small equal entries and a
    # balancing entry, all exactly representable; the pair is (phi, phi)
    small = 2.0 ** -12 * (1 - 2.0 ** -8)
    comps = np.array([0.75] + [small] * 126 + [0.0])
    comps[-1] = oracle.round_to_bf16(np.array([math.sqrt(1.0 - math.fsum((comps[:-1] ** 2).tolist()))]))[0]
    nrm = math.sqrt(math.fsum((comps ** 2).tolist()))
    phi = comps[0::2] + 1j * comps[1::2]
    g_exact = math.fsum((comps ** 2).tolist())
    g_trunc = screened_inner(phi, phi, "zero").real
    err = g_exact - g_trunc
    eps = oracle.screen_error_bound(d)
    no_accumulation = 8 * 2.0 ** -24 + 1e-12            # input term is 0 here: exact bf16 inputs
    assert abs(nrm - 1.0) < 2 * U                        # a unit column up to the balancing entry's rounding
    assert err > no_accumulation
    assert err <= eps


@pytest.mark.parametrize("direction", ["nearest", "zero", "up", "down"])
def test_adversarial_frame_with_directed_accumulation_within_bound(direction):
    d = 64
    phi, psi = adversarial_pair(d)
    F = np.stack([phi, psi], axis=1)
    exact = oracle.coherence(F)
    g = screened_inner(_rounded(phi), _rounded(psi), direction)
    screen = math.sqrt(g.real * g.real + g.imag * g.imag)
    assert abs(screen - exact) <= oracle.screen_error_bound(d)
    assert abs(screen - exact) >= 0.93 * 2 * U


@pytest.mark.parametrize("direction", ["zero", "up"])
def test_random_frames_with_directed_accumulation_within_bound(direction):
    rng = np.random.default_rng(7)
    for d in (3, 32, 64):
        Z = rng.standard_normal((d, 6)) + 1j * rng.standard_normal((d, 6))
        F, _ = oracle.normalize_columns(Z)
        R = _rounded(F)
        eps = oracle.screen_error_bound(d)
        G = F.conj().T @ F
        for j in range(6):
            for k in range(j + 1, 6):
                g = screened_inner(R[:, j], R[:, k], direction)
                assert abs(abs(g) - abs(G[j, k])) <= eps


def test_bound_value_and_growth():
    """The bound is the input term plus terms that grow with d: at d = 64,
    2u + u^2 = 0.0078278 plus sqrt(2) gamma_128(2^-23) (1 + u)^2 = 2.17e-5 and
    the epilogue."""
    e64 = oracle.screen_error_bound(64)
    base = 2 * U + U * U
    acc = math.sqrt(2) * (128 * W / (1 - 128 * W)) * (1 + U) ** 2
    assert abs(e64 - (base + acc + 8 * 2.0 ** -24 + 1e-12)) < 1e-18
    assert 2.1e-5 < acc < 2.2e-5
    assert oracle.screen_error_bound(128) > e64 > oracle.screen_error_bound(16)
