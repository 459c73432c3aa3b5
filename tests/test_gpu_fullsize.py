"""GPU parity at the workload sizes themselves, through the C ABI.

* The throughput step: N = 4096 unit vectors in C^64, C = 128 candidates,
  radius 0.05, BF16 screen with the top 8 rechecked in FP64 (Haar start,
  seed 0).  Each test runs one oracle step (about 40 s of CPU): every screened
  value against the oracle's BF16 emulation, the rechecked set, the rechecked
  candidates' FP64 coherence (definition of mu, section I; only the upper
  triangle of |G|, section IV) and the decision, radius, mu and frame.
* The plain step: N = 1024 in C^32, C = 256, radius 0.05, FP64 and FP32.
"""

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lib = pytest.importorskip("paper_2207_06374_amd")

MAX_STEPS = 2 ** 32 - 1


def _pair(n, d, C, mode, radius0, k=8):
    s = lib.Solver(n, d, candidates=C, mode=mode, radius0=radius0, max_steps=MAX_STEPS, seed=0, recheck_topk=k)
    p = oracle.Params(n=n, d=d, candidates=C, mode=mode, radius0=radius0, max_steps=MAX_STEPS, seed=0,
                      recheck_topk=k)
    return s, p


def _sync_oracle(s, p):
    F, mu, radius, t, flags = s.host_state()
    return oracle.State(frame=F, mu=mu, radius=radius, t=t, done=bool(flags & lib.FLAG_DONE))


@pytest.mark.parametrize("t_start", [0, 1])
def test_headline_bf16_step_full_size(t_start):
    n, d, C, k = 4096, 64, 128, 8
    print(f"headline step parity: N={n} d={d} C={C} k={k} step {t_start}", flush=True)
    s, p = _pair(n, d, C, "bf16", 0.05, k)
    s.init_haar()
    if t_start == 0:
        ref0 = oracle.haar_init(p)
        F0, mu0, r0, t0, fl0 = s.host_state()
        assert np.max(np.abs(F0 - ref0.frame)) <= 1e-14
        assert abs(mu0 - ref0.mu) <= 1e-12 and r0 == 0.05 and t0 == 0 and fl0 == 0
    for _ in range(t_start):
        s.step(with_report=False)
    st = _sync_oracle(s, p)
    assert st.t == t_start and not st.done
    s.step()
    F, mu, radius, tt, flags = s.host_state()
    screened = s.report["cand_mu"].cpu().numpy()
    rechecked = s.report["rechecked"].cpu().numpy()[:k].astype(np.int64)
    recheck_mu = s.report["recheck_mu"].cpu().numpy()[:k]
    best = int(s.report["best"].item())

    new, rep = oracle.step(p, st, exact_all=False)
    eps = oracle.screen_error_bound(d)
    # every screened value: the same bf16 inputs as the oracle's emulation, only
    # the FP32 accumulation differs
    assert np.max(np.abs(screened - rep.cand_mu)) <= 2e-5
    # the GPU rechecked exactly its own k best screened values ...
    order = sorted(range(C), key=lambda c: (screened[c], c))
    assert list(rechecked) == order[:k]
    # ... and their FP64 coherences are exact (the oracle evaluates the same candidates)
    Z = oracle.perturbations(p, st.t, cands=rechecked)
    Phi_c, valid = oracle.make_candidates(st.frame, st.radius, d, Z)
    exact = oracle.evaluate_candidates(Phi_c, valid, "fp64")
    assert np.max(np.abs(recheck_mu - exact)) <= 1e-12
    assert np.max(np.abs(screened[rechecked] - exact)) <= eps
    print(f"  screen-emulation max diff {np.max(np.abs(screened - rep.cand_mu)):.3e}, "
          f"screen-exact max diff {np.max(np.abs(screened[rechecked] - exact)):.3e}, eps {eps:.5f}", flush=True)
    assert tt == t_start + 1
    # the decision follows from the GPU's own exact values: c* = argmin over
    # (mu, c) in the rechecked set, accept iff mu_{c*} < mu_t, radius x2 / x0.5
    i_best = min(range(k), key=lambda i: (recheck_mu[i], rechecked[i]))
    assert best == rechecked[i_best]
    accepted = bool(recheck_mu[i_best] < st.mu)
    assert bool(flags & lib.FLAG_ACCEPTED) == accepted
    assert radius == (min(2 * st.radius, 1.0) if accepted else max(st.radius / 2, 1e-12))
    if accepted:
        assert mu == recheck_mu[i_best]
    if rep.near_tie or (flags & lib.FLAG_NEAR_TIE):
        print(f"  near tie at step {t_start} (screen gap {rep.screen_gap:.3e}): the oracle's decision may differ",
              flush=True)
        return
    assert list(rechecked) == list(rep.rechecked)
    assert best == rep.best
    assert bool(flags & lib.FLAG_ACCEPTED) == rep.accepted
    assert radius == new.radius
    assert abs(mu - new.mu) <= 1e-12
    assert np.max(np.abs(F - new.frame)) <= 1e-13


@pytest.mark.parametrize("mode", ["fp64", "fp32"])
def test_plain_step_full_size(mode):
    n, d, C = 1024, 32, 256
    print(f"plain step parity: N={n} d={d} C={C} {mode}", flush=True)
    s, p = _pair(n, d, C, mode, 0.05)
    s.init_haar()
    if mode == "fp64":
        ref0 = oracle.haar_init(p)
        F0, mu0, _, _, _ = s.host_state()
        assert np.max(np.abs(F0 - ref0.frame)) <= 1e-14 and abs(mu0 - ref0.mu) <= 1e-12
    for t in range(2):
        st = _sync_oracle(s, p)
        s.step()
        new, rep = oracle.step(p, st)
        F, mu, radius, tt, flags = s.host_state()
        cand = s.report["cand_mu"].cpu().numpy()
        if mode == "fp64":
            assert np.max(np.abs(cand - rep.cand_mu)) <= 1e-12, f"step {t}"
        else:
            assert np.max(np.abs(cand - rep.cand_mu_fp64)) <= 2e-6, f"step {t}"
            assert np.max(np.abs(cand - rep.cand_mu)) <= 1e-6, f"step {t}"
        if rep.near_tie or (flags & lib.FLAG_NEAR_TIE):
            continue
        assert int(s.report["best"].item()) == rep.best
        assert bool(flags & lib.FLAG_ACCEPTED) == rep.accepted
        assert radius == new.radius and tt == new.t
        if mode == "fp64" or rep.accepted:
            assert abs(mu - new.mu) <= (1e-12 if mode == "fp64" else 2e-6)
        if rep.accepted:
            assert np.max(np.abs(F - new.frame)) <= 1e-13
