"""Pins for the oracle's candidate search: step, accept/radius rule, forms."""

import math

import numpy as np
import pytest

import frames
import inputs
import oracle


def _params(**kw):
    base = dict(n=16, d=4, candidates=16, mode="fp64", seed=0, radius0=0.1, max_steps=50)
    base.update(kw)
    return oracle.Params(**base)


def test_haar_start_is_unit_and_deterministic():
    p = _params()
    a, b = oracle.haar_init(p), oracle.haar_init(p)
    assert np.array_equal(a.frame, b.frame) and a.mu == b.mu
    assert np.allclose(np.linalg.norm(a.frame, axis=0), 1, atol=1e-15)
    assert abs(a.mu - oracle.coherence(a.frame)) <= 1e-15
    assert a.radius == 0.1 and a.t == 0


def test_candidates_are_unit_and_centered_on_frame():
    p = _params(n=40, d=6)
    st = oracle.haar_init(p)
    Z = oracle.perturbations(p, 0)
    assert Z.shape == (16, 6, 40)
    C, valid = oracle.make_candidates(st.frame, 1e-9, p.d, Z)
    assert valid.all()
    assert np.allclose(np.linalg.norm(C, axis=1), 1, atol=1e-15)
    assert np.max(np.abs(C - st.frame[None])) < 1e-8   # tiny radius -> candidates close to frame
    # RMS column displacement is about the radius
    C2, _ = oracle.make_candidates(st.frame, 0.01, p.d, Z)
    Y = st.frame[None] + 0.01 / math.sqrt(6) * Z
    rms = np.sqrt(np.mean(np.sum(np.abs(Y - st.frame[None]) ** 2, axis=1)))
    assert 0.008 < rms < 0.012


def test_known_winner_accepted_and_radius_grows():
    """Candidate 0 is steered onto the d=2 SIC, the best possible 4 lines: it
    must be selected and accepted, and the radius must double."""
    p = _params(n=4, d=2, candidates=8, radius0=0.25)
    st = oracle.haar_init(p)
    s = st.radius / math.sqrt(p.d)
    Z = inputs.random_perturbation(4, 2, 8, seed=1)
    Z[0] = (frames.tetrahedron_c2() - st.frame) / s
    new, rep = oracle.step(p, st, Z)
    assert rep.best == 0 and rep.accepted
    assert abs(new.mu - 1 / math.sqrt(3)) <= 1e-14
    assert new.radius == 0.5 and new.t == 1
    assert np.all(rep.cand_mu[1:] > rep.cand_mu[0])


def test_reject_shrinks_radius_and_keeps_frame():
    p = _params(n=4, d=2, candidates=4, radius0=0.25)
    st = oracle.haar_init(p)
    st.frame = frames.tetrahedron_c2()
    st.mu = oracle.coherence(st.frame)
    new, rep = oracle.step(p, st)
    assert not rep.accepted                    # nothing beats the Welch bound
    assert np.array_equal(new.frame, st.frame) and new.mu == st.mu
    assert new.radius == 0.125


def test_ties_go_to_lowest_index_and_invalid_never_wins():
    p = _params(n=6, d=3, candidates=5, radius0=0.3)
    st = oracle.haar_init(p)
    Z = inputs.random_perturbation(6, 3, 5, seed=2)
    _, rep0 = oracle.step(p, st, Z)
    w = rep0.best
    # the winner duplicated at index 4 and the lowest other index: lowest index wins
    lo = 0 if w != 0 else 1
    Z2 = Z.copy()
    Z2[4] = Z[w]
    Z2[lo] = Z[w]
    _, rep = oracle.step(p, st, Z2)
    assert rep.best == min(lo, w)
    # a non-finite perturbation makes that candidate invalid: mu = inf, never chosen
    Z3 = Z2.copy()
    Z3[rep.best][1, 2] = np.nan
    _, rep3 = oracle.step(p, st, Z3)
    assert not rep3.valid[rep.best] and rep3.cand_mu[rep.best] == math.inf
    assert rep3.best == min(i for i in (lo, w, 4) if i != rep.best)


def test_zero_perturbation_is_a_logged_near_tie():
    p = _params(n=10, d=3, candidates=4)
    st = oracle.haar_init(p)
    Z = np.zeros((4, 3, 10), dtype=np.complex128)
    _, rep = oracle.step(p, st, Z)
    assert rep.near_tie
    assert np.all(np.abs(rep.cand_mu - st.mu) <= 1e-15)


def test_radius_clamps():
    p = _params(radius0=1.0, radius_max=1.0)
    st = oracle.haar_init(p)
    st.frame = frames.sic_numeric(4)
    st.mu = oracle.coherence(st.frame)
    st.radius = 1e-12
    new, rep = oracle.step(_params(radius_min=1e-12), st)
    assert not rep.accepted and new.radius == 1e-12
    p2 = _params(n=4, d=2, candidates=2, radius0=1.0)
    st2 = oracle.haar_init(p2)
    Z = inputs.random_perturbation(4, 2, 2, seed=3)
    Z[0] = (frames.tetrahedron_c2() - st2.frame) / (1.0 / math.sqrt(2))
    new2, rep2 = oracle.step(p2, st2, Z)
    assert rep2.accepted and new2.radius == 1.0


def test_solve_small_is_monotone_and_on_radius_lattice():
    p = _params(candidates=64, max_steps=200)
    st, hist = oracle.solve(p, record=True)
    mus = [h[1] for h in hist]
    assert all(b <= a for a, b in zip(mus, mus[1:]))
    assert st.mu >= oracle.welch_bound(16, 4) - 1e-12
    assert st.t == 200 and st.done
    for _, _, r, _, _ in hist:
        k = math.log2(r / 0.1)
        assert r in (1e-12, 1.0) or abs(k - round(k)) < 1e-12
    assert abs(st.mu - oracle.coherence(st.frame)) <= 1e-15
    assert st.mu < oracle.haar_init(p).mu


def test_resume_equivalence():
    p = _params(max_steps=40)
    full, _ = oracle.solve(p)
    half, _ = oracle.solve(_params(max_steps=20))
    half.done = False
    rest, _ = oracle.solve(p, state=half)
    assert np.array_equal(full.frame, rest.frame) and full.mu == rest.mu and full.radius == rest.radius


def test_target_stops_early():
    p = _params(max_steps=500, target_mu=0.9)
    st, hist = oracle.solve(p, record=True)
    assert st.mu <= 0.9 and st.t < 500


def test_fp32_form_close_to_fp64():
    p = _params(n=64, d=8, candidates=12, mode="fp32")
    st = oracle.haar_init(p)
    _, rep = oracle.step(p, st)
    assert np.max(np.abs(rep.cand_mu - rep.cand_mu_fp64)) <= 2e-6
    assert np.any(rep.cand_mu != rep.cand_mu_fp64)


@pytest.mark.parametrize("n,d", [(64, 8), (200, 16), (96, 32)])
def test_bf16_screen_within_bound_and_recheck_exact(n, d):
    p = _params(n=n, d=d, candidates=24, mode="bf16", recheck_topk=5, radius0=0.2)
    st = oracle.haar_init(p)
    _, rep = oracle.step(p, st)
    eps = oracle.screen_error_bound(d)
    assert 0.00782 < eps < 0.00786
    err = np.abs(rep.cand_mu - rep.cand_mu_fp64)
    assert np.max(err) <= eps
    assert np.max(err) > 1e-5                              # rounding really happened
    assert len(rep.rechecked) == 5 and rep.best in rep.rechecked
    order = sorted(range(24), key=lambda c: (rep.cand_mu[c], c))
    assert list(rep.rechecked) == order[:5]
    assert rep.best_mu == rep.cand_mu_fp64[rep.best]
    assert rep.best_mu == min(rep.cand_mu_fp64[rep.rechecked])
    # the chosen candidate is within 2 eps of the true best over all C
    assert rep.best_mu <= np.min(rep.cand_mu_fp64) + 2 * eps


def test_bf16_topk_all_equals_fp64_choice():
    p = _params(n=30, d=5, candidates=10, mode="bf16", recheck_topk=10)
    p64 = _params(n=30, d=5, candidates=10, mode="fp64")
    st = oracle.haar_init(p64)
    a, ra = oracle.step(p, st)
    b, rb = oracle.step(p64, st)
    assert ra.best == rb.best and a.mu == b.mu and np.array_equal(a.frame, b.frame)


def test_accept_is_strict():
    """A best candidate exactly equal to the current coherence is rejected."""
    p = _params(n=12, d=3, candidates=6)
    st = oracle.haar_init(p)
    Z = oracle.perturbations(p, 0)
    _, rep = oracle.step(p, st, Z)
    st2 = st.copy()
    st2.mu = rep.best_mu
    new, rep2 = oracle.step(p, st2, Z)
    assert rep2.best == rep.best and not rep2.accepted and rep2.near_tie
    assert new.radius == st.radius * 0.5
    st2.mu = np.nextafter(rep.best_mu, 1.0)
    _, rep3 = oracle.step(p, st2, Z)
    assert rep3.accepted


def test_bf16_exact_all_false_changes_no_decision():
    """exact_all=False skips the FP64 values no decision reads: the same
    rechecked set, choice, frame, radius and FP64 values of the rechecked."""
    p = _params(n=64, d=8, candidates=24, mode="bf16", recheck_topk=5, radius0=0.2)
    st = oracle.haar_init(p)
    for _ in range(3):
        a, ra = oracle.step(p, st)
        b, rb = oracle.step(p, st, exact_all=False)
        assert ra.best == rb.best and ra.accepted == rb.accepted and ra.near_tie == rb.near_tie
        assert a.mu == b.mu and a.radius == b.radius and np.array_equal(a.frame, b.frame)
        assert np.array_equal(ra.rechecked, rb.rechecked)
        assert np.array_equal(ra.cand_mu, rb.cand_mu)
        assert np.array_equal(ra.cand_mu_fp64[ra.rechecked], rb.cand_mu_fp64[rb.rechecked])
        assert np.isnan(rb.cand_mu_fp64).sum() == 24 - 5
        st = a
