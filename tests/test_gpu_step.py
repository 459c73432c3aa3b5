"""GPU parity: trstmi_step / trstmi_solve against the oracle's step."""

import math

import numpy as np
import pytest

import frames
import inputs
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lib = pytest.importorskip("paper_2207_06374_amd")


def _pair(n, d, C, mode="fp64", radius0=0.1, max_steps=1000, seed=0, k=8, **kw):
    s = lib.Solver(n, d, candidates=C, mode=mode, radius0=radius0, max_steps=max_steps, seed=seed,
                   recheck_topk=k, **kw)
    p = oracle.Params(n=n, d=d, candidates=C, mode=mode, radius0=radius0, max_steps=max_steps, seed=seed,
                      recheck_topk=k, **kw)
    return s, p


def _sync_oracle(s, p):
    F, mu, radius, t, flags = s.host_state()
    return oracle.State(frame=F, mu=mu, radius=radius, t=t, done=bool(flags & lib.FLAG_DONE))


@pytest.mark.parametrize("n,d,C", [(16, 4, 64), (70, 5, 16), (200, 16, 32), (130, 33, 8)])
def test_fp64_trajectory_parity(n, d, C):
    """FP64: the GPU trajectory follows the oracle's step by step (no resync)
    until a logged near tie."""
    s, p = _pair(n, d, C, radius0=0.1)
    s.init_haar()
    st = oracle.haar_init(p)
    steps = 60 if n <= 70 else 12
    for t in range(steps):
        s.step()
        new, rep = oracle.step(p, st)
        F, mu, radius, tt, flags = s.host_state()
        cand = s.report["cand_mu"].cpu().numpy()
        best = int(s.report["best"].item())
        assert np.max(np.abs(cand - rep.cand_mu)) <= 1e-12, f"step {t}"
        if rep.near_tie or (flags & lib.FLAG_NEAR_TIE):
            print(f"near tie at step {t}; stopping trajectory comparison", flush=True)
            return
        assert best == rep.best, f"step {t}"
        assert bool(flags & lib.FLAG_ACCEPTED) == rep.accepted
        assert radius == new.radius and tt == new.t
        assert abs(mu - new.mu) <= 1e-12
        assert np.max(np.abs(F - new.frame)) <= 1e-13
        st = new


@pytest.mark.parametrize("n,d,C", [(16, 4, 64), (100, 8, 24), (300, 32, 16)])
def test_fp32_step_parity_with_resync(n, d, C):
    s, p = _pair(n, d, C, mode="fp32", radius0=0.1)
    s.init_haar()
    st0 = _sync_oracle(s, p)
    ref0 = oracle.haar_init(p)
    assert abs(st0.mu - oracle.coherence(st0.frame)) <= 2e-6
    assert abs(st0.mu - ref0.mu) <= 2e-6
    for t in range(10):
        st = _sync_oracle(s, p)
        s.step()
        new, rep = oracle.step(p, st)
        F, mu, radius, tt, flags = s.host_state()
        cand = s.report["cand_mu"].cpu().numpy()
        assert np.max(np.abs(cand - rep.cand_mu_fp64)) <= 2e-6
        assert np.max(np.abs(cand - rep.cand_mu)) <= 1e-6
        if rep.near_tie or (flags & lib.FLAG_NEAR_TIE):
            continue
        assert int(s.report["best"].item()) == rep.best
        assert bool(flags & lib.FLAG_ACCEPTED) == rep.accepted
        assert radius == new.radius
        if rep.accepted:
            assert np.max(np.abs(F - new.frame)) <= 1e-13


@pytest.mark.parametrize("n,d,C,k", [(64, 8, 32, 4), (300, 16, 24, 8), (260, 64, 16, 8), (129, 3, 40, 8),
                                     (16, 4, 1100, 8)])
def test_bf16_screen_step_parity(n, d, C, k):
    s, p = _pair(n, d, C, mode="bf16", k=k, radius0=0.2)
    s.init_haar()
    eps = oracle.screen_error_bound(d)
    for t in range(6):
        st = _sync_oracle(s, p)
        s.step()
        new, rep = oracle.step(p, st)
        F, mu, radius, tt, flags = s.host_state()
        screened = s.report["cand_mu"].cpu().numpy()
        rechecked = s.report["rechecked"].cpu().numpy()[:k]
        recheck_mu = s.report["recheck_mu"].cpu().numpy()[:k]
        # every screened value within the certified bound of the exact FP64 value
        assert np.max(np.abs(screened - rep.cand_mu_fp64)) <= eps
        # same bf16 inputs as the oracle's emulation: only FP32 accumulation differs
        assert np.max(np.abs(screened - rep.cand_mu)) <= 2e-5
        # the GPU rechecked exactly its own k best screened values, and their FP64 values are exact
        order = sorted(range(C), key=lambda c: (screened[c], c))
        assert list(rechecked) == order[:k]
        assert np.max(np.abs(recheck_mu - rep.cand_mu_fp64[rechecked])) <= 1e-12
        if rep.near_tie or (flags & lib.FLAG_NEAR_TIE):
            continue
        assert list(rechecked) == list(rep.rechecked)
        assert int(s.report["best"].item()) == rep.best
        assert bool(flags & lib.FLAG_ACCEPTED) == rep.accepted
        assert radius == new.radius
        assert abs(mu - new.mu) <= 1e-12
        assert np.max(np.abs(F - new.frame)) <= 1e-13


def test_bf16_recheck_with_many_near_maximal_pairs():
    """Candidates near an equiangular frame (Hesse SIC, 9 lines in C^3): every
    pair lies within the screen's error band of the maximum, so the FP64
    recheck evaluates many pairs per tile (both its one-pair-per-wave and its
    one-pair-per-lane paths) and must still return the exact FP64 values."""
    F0 = frames.hesse_sic()
    n, d, C, k = 9, 3, 16, 8
    s, p = _pair(n, d, C, mode="bf16", k=k, radius0=1e-3)
    s.set_frame(F0, mu=oracle.coherence(F0), radius=1e-3)
    for _ in range(3):
        st = _sync_oracle(s, p)
        s.step()
        new, rep = oracle.step(p, st)
        rechecked = s.report["rechecked"].cpu().numpy()[:k]
        recheck_mu = s.report["recheck_mu"].cpu().numpy()[:k]
        assert np.max(np.abs(recheck_mu - rep.cand_mu_fp64[rechecked])) <= 1e-12


def test_known_winner_through_abi():
    n, d, C = 4, 2, 8
    s, p = _pair(n, d, C, radius0=0.25)
    s.init_haar()
    st = _sync_oracle(s, p)
    sc = st.radius / math.sqrt(d)
    Z = inputs.random_perturbation(n, d, C, seed=1)
    Z[0] = (frames.tetrahedron_c2() - st.frame) / sc
    zdev = torch.from_numpy(np.ascontiguousarray(np.transpose(Z, (0, 2, 1))).view(np.float64).ravel().copy()).cuda()
    s.step(explicit_z=zdev)
    F, mu, radius, t, flags = s.host_state()
    assert int(s.report["best"].item()) == 0 and flags & lib.FLAG_ACCEPTED
    assert abs(mu - 1 / math.sqrt(3)) <= 1e-12 and radius == 0.5 and t == 1
    assert abs(oracle.coherence(F) - 1 / math.sqrt(3)) <= 1e-12


def test_done_state_is_noop_and_target_stops():
    s, p = _pair(16, 4, 16, max_steps=3)
    s.init_haar()
    for _ in range(5):
        s.step()
    F, mu, radius, t, flags = s.host_state()
    assert t == 3 and flags & lib.FLAG_DONE
    s2, _ = _pair(16, 4, 16, max_steps=500, target_mu=0.9)
    s2.init_haar()
    s2.solve(chunk=7)
    F, mu, radius, t, flags = s2.host_state()
    assert mu <= 0.9 and flags & lib.FLAG_DONE and t < 500


@pytest.mark.parametrize("mode", ["fp64", "bf16"])
def test_small_solve_matches_oracle(mode):
    """The small workload (N=16 in C^4, 64 candidates, radius 0.1, 2000 steps)
    solved on the GPU with graph-captured chunks follows the oracle's
    trajectory.  The run is cut into segments at the oracle's near-tie
    decisions: between two of them the GPU solve must reach the oracle's
    state (frame, mu, radius, step); the near-tie step itself is taken by the
    GPU alone and the oracle resyncs to its state."""
    total = 2000
    s, p = _pair(16, 4, 64, mode=mode, radius0=0.1, max_steps=total, k=8)
    s.init_haar()
    st = oracle.haar_init(p)
    F0, mu0, _, _, _ = s.host_state()
    assert np.max(np.abs(F0 - st.frame)) <= 1e-14 and abs(mu0 - st.mu) <= 1e-12
    segments = ties = solved_steps = 0
    mus = [mu0]
    while True:
        ost, stop = st, total
        while ost.t < total:
            nxt, rep = oracle.step(p, ost, exact_all=False)
            if rep.near_tie:
                stop = ost.t
                break
            ost = nxt
        if stop > st.t:
            s.params.max_steps = stop
            s.state.flags.fill_(0)
            s.solve(chunk=64)
            segments += 1
            solved_steps += stop - st.t
        F, mu, radius, t, flags = s.host_state()
        assert t == stop, f"segment ending at {stop}"
        assert abs(mu - ost.mu) <= 1e-12, f"step {stop}"
        assert radius == ost.radius, f"step {stop}"
        assert np.max(np.abs(F - ost.frame)) <= 1e-12, f"step {stop}"
        mus.append(mu)
        if stop >= total:
            break
        s.params.max_steps = total
        s.state.flags.fill_(0)
        s.step(with_report=False)
        ties += 1
        st = _sync_oracle(s, p)
        mus.append(st.mu)
    F, mu, radius, t, flags = s.host_state()
    print(f"{mode}: {segments} solve segments ({solved_steps} steps), {ties} near-tie steps", flush=True)
    assert t == total and flags & lib.FLAG_DONE
    assert all(b <= a for a, b in zip(mus, mus[1:]))       # mu never increases
    assert mu >= oracle.welch_bound(16, 4) - 1e-12
    assert solved_steps > 0


def test_step_matches_solve_bitwise():
    a, _ = _pair(40, 6, 16, max_steps=25)
    b, _ = _pair(40, 6, 16, max_steps=25)
    a.init_haar()
    b.init_haar()
    for _ in range(25):
        a.step(with_report=False)
    b.solve(chunk=8)
    A, B = a.host_state(), b.host_state()
    assert np.array_equal(A[0], B[0]) and A[1:] == B[1:]
