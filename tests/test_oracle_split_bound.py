"""Pins of the batched form's split-screen error bound
(``oracle.split_screen_error_bound``).

The batched form screens each candidate with every real component held as two
bfloat16 parts (hi + lo of its binary32 rounding) and three products per real
pair (hi hi' + hi lo' + lo hi') accumulated in binary32, and rechecks in FP64
only the pairs whose screened |G| lies within twice the bound of the screened
maximum.  That recheck finds the exact maximum only if |screened - exact|
never exceeds the bound.  These tests check the pieces of the bound and the
bound itself against inputs built to make the errors add up:

* the representation: hi + lo is within 2^-17 of the binary32 value (the
  remainder lies at least nine binades below it), the remainder f - hi is
  exact, and random values come close to 2^-17 (the term is nearly tight);
* an adversarial pair whose components all carry a near-largest
  representation error, arranged so that every such error raises
  Re<phi, psi>: it reaches a clear part of the input term, exceeds the bound
  of a plain binary32 screen, and stays within the full bound under every
  rounding direction of the accumulation;
* random frames under directed accumulation stay within the bound.

The screen emulation here is a test helper written from the description
above (products of bfloat16 values are exact in FP64; each binary32 addition
is emulated from the exact FP64 sum).
"""

import math

import numpy as np
import pytest

import oracle

U = 2.0 ** -8
V = 2.0 ** -24


def split(f):
    """(hi, lo) of binary32 values f (given as float64 holding binary32
    values): hi = bf16(f), lo = bf16(f - hi), both round to nearest even."""
    f = np.asarray(f, dtype=np.float64)
    hi = oracle.round_to_bf16(f)
    r = f - hi                          # exact in FP64 (and in binary32)
    return hi, oracle.round_to_bf16(r)


def reals(z):
    out = np.empty(2 * z.size)
    out[0::2], out[1::2] = z.real, z.imag
    return out


def rotated(z):
    """Reals of (Im, -Re) per entry: the second operand of Im<phi, psi>."""
    out = np.empty(2 * z.size)
    out[0::2], out[1::2] = z.imag, -z.real
    return out


def fp32_sum(terms, direction):
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


def split_dot(a, b, direction):
    """Binary32 accumulation of hi lo', lo hi' and hi hi' over the reals a, b
    (binary32-rounded first), in that order."""
    ha, la = split(np.float32(a).astype(np.float64))
    hb, lb = split(np.float32(b).astype(np.float64))
    terms = np.concatenate([ha * lb, la * hb, ha * hb])
    return fp32_sum(terms, direction)


def screened(phi, psi, direction="nearest"):
    re = split_dot(reals(phi), reals(psi), direction)
    im = split_dot(reals(phi), rotated(psi), direction)
    g2 = np.float32(np.float32(re) * np.float32(re) + np.float32(im) * np.float32(im))
    return math.sqrt(float(g2))


def test_representation_is_exact_remainder_and_within_2_pow_minus_17():
    rng = np.random.default_rng(3)
    f = np.float32(rng.standard_normal(200000) * np.exp2(rng.integers(-20, 4, 200000))).astype(np.float64)
    hi, lo = split(f)
    r = f - hi
    assert np.array_equal(np.float32(r).astype(np.float64), r)          # the remainder is binary32-exact
    rel = np.abs(hi + lo - f) / np.abs(f)
    assert rel.max() <= 2.0 ** -17
    assert np.all(np.abs(r) <= U * np.abs(f)) and np.all(np.abs(lo) <= U * (1 + U) * np.abs(f))
    # random values come close to 2^-17 ...
    assert rel.max() >= 0.9 * 2.0 ** -17
    # ... and a bound of half of it would be wrong
    assert rel.max() > 0.5 * 2.0 ** -17


def _extreme_pools(seed=0):
    """binary32 values in [0.06, 0.6] whose relative representation error
    (hi + lo - f) / f is at least 0.8 x 2^-17 upwards and downwards (they sit
    just above powers of two)."""
    rng = np.random.default_rng(seed)
    f = np.float32(rng.uniform(0.06, 0.6, 2000000)).astype(np.float64)
    hi, lo = split(f)
    e = (hi + lo - f) / f
    return np.unique(f[e >= 0.8 * 2.0 ** -17]), np.unique(f[e <= -0.8 * 2.0 ** -17])


def _greedy(pools, kinds, total):
    """One value per entry of ``kinds`` (0: pools[0], 1: pools[1]), each the
    unused value nearest to the root of the remaining budget over the
    remaining slots, so that the squares add up to about ``total``."""
    used = [np.zeros(p.size, dtype=bool) for p in pools]
    out = []
    for i, k in enumerate(kinds):
        left = total - math.fsum([v * v for v in out])
        want = math.sqrt(max(left, 0.0) / (len(kinds) - i))
        dist = np.where(used[k], np.inf, np.abs(pools[k] - want))
        j = int(np.argmin(dist))
        used[k][j] = True
        out.append(float(pools[k][j]))
    return np.array(out)


def adversarial_pair(d):
    """Columns phi, psi in C^d (unit to about 1e-7) with equal component
    moduli.  The first d - 1 complex entries (2d - 2 reals) carry extreme
    representation errors: "agree" entries (the same sign in phi and psi, a
    majority, so that Re<phi, psi> > 0) err upwards, "disagree" entries
    (opposite signs) downwards, so that every error raises Re<phi~, psi~> by
    about 2 x 2^-17 of its share; the real and imaginary parts of one entry
    share their group, so Im<phi, psi> = 0.  One
    more real (squared about 0.05) brings the norm to 1.  The columns are
    binary32 values already, so only the split moves them."""
    up, down = _extreme_pools()
    m = 2 * d - 2
    n_up = 2 * ((d - 1) // 2 + 1)                  # reals in agree entries: whole entries, a majority
    # alternate the groups in the draw so that both get values of the same sizes
    kinds = [0, 1] * (m - n_up) + [0] * (2 * n_up - m)
    vals = _greedy((up, down), kinds, 0.95)
    kinds = np.array(kinds)
    x = np.concatenate([vals[kinds == 0], vals[kinds == 1]])
    t2 = 1.0 - math.fsum((x * x).tolist())
    assert 0.01 <= t2 <= 0.12
    comps = np.zeros(2 * d)
    comps[:m] = x
    comps[m] = float(np.float32(math.sqrt(t2)))   # comps[m + 1] (its partner) stays 0
    signs = np.ones(2 * d)
    signs[n_up:m] = -1.0
    phi = comps[0::2] + 1j * comps[1::2]
    psi = (comps * signs)[0::2] + 1j * (comps * signs)[1::2]
    # left as they are: dividing by the FP64 norm would move every component
    # off the binary32 values chosen above
    assert abs(np.linalg.norm(phi) - 1.0) < 1e-7 and abs(np.linalg.norm(psi) - 1.0) < 1e-7
    return phi, psi


@pytest.mark.parametrize("d", [6, 16])
def test_adversarial_pair_reaches_the_input_term_and_stays_within_bound(d):
    phi, psi = adversarial_pair(d)
    exact = abs(np.vdot(phi, psi))                 # the columns as given (unit to 1e-7)
    assert abs(np.vdot(phi, psi).imag) < 1e-15
    eps = oracle.split_screen_error_bound(d)
    errs = {dirn: screened(phi, psi, dirn) - exact for dirn in ("nearest", "zero", "up", "down")}
    for dirn, err in errs.items():
        assert abs(err) <= eps, dirn
    err = errs["nearest"]
    # most of the input term 2 delta (about 1.54e-5) is attained (the dropped
    # lo lo' of the majority group take some of it back) ...
    assert err >= 0.5 * 2 * 2.0 ** -17
    # ... which the binary32 screen's own bound (inputs rounded to binary32,
    # 2d products per part) does not cover
    w = 2.0 ** -23
    fp32_bound = 2 * V + V * V + math.sqrt(2) * (2 * d * w / (1 - 2 * d * w)) * (1 + V) ** 2 + 16 * V + 1e-12
    assert err > fp32_bound


@pytest.mark.parametrize("direction", ["zero", "up"])
def test_random_frames_with_directed_accumulation_within_bound(direction):
    rng = np.random.default_rng(11)
    for d in (3, 9, 16):
        Z = rng.standard_normal((d, 5)) + 1j * rng.standard_normal((d, 5))
        F, _ = oracle.normalize_columns(Z)
        G = F.conj().T @ F
        eps = oracle.split_screen_error_bound(d)
        for j in range(5):
            for k in range(j + 1, 5):
                assert abs(screened(F[:, j], F[:, k], direction) - abs(G[j, k])) <= eps


def test_bound_value():
    """About 5.45e-5: the input term 2 delta = 1.54e-5, sqrt 2 times the
    dropped products 1.54e-5 and the accumulation 1.16e-5, and the epilogue;
    the same for every d <= 16 (the reals are padded to 32); refused above."""
    e = oracle.split_screen_error_bound(16)
    delta = 2.0 ** -17 * (1 + V) + V
    assert 1.53e-5 < 2 * delta < 1.55e-5
    assert 5.4e-5 < e < 5.5e-5
    assert oracle.split_screen_error_bound(3) == e
    # about ten times the binary32 screen's, far below the bfloat16 one's
    assert 8 * (2 * V + math.sqrt(2) * 32 * 2.0 ** -23) < e < oracle.screen_error_bound(16) / 100
    with pytest.raises(ValueError):
        oracle.split_screen_error_bound(17)
