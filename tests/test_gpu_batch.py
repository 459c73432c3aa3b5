"""GPU parity of the batched form: every instance follows the FP64 oracle
search with its own stream, and does not depend on the rest of the batch or on
its waves-per-item tile choice."""

import numpy as np
import pytest

import inputs
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lib = pytest.importorskip("paper_2207_06374_amd")
autotune = pytest.importorskip("paper_2207_06374_amd.autotune")


def _specs(count, seed, d_hi=8, max_steps=1000, wpi=0, d_lo=3):
    out = []
    for k, (d, n) in enumerate(inputs.batched_instances(count, seed=seed, d_lo=d_lo, d_hi=d_hi)):
        out.append({"n": n, "d": d, "seed": 7, "stream_id": 100 + k, "max_steps": max_steps, "waves_per_item": wpi})
    return out


def _oracle_params(spec, C, radius0=0.1):
    return oracle.Params(n=spec["n"], d=spec["d"], candidates=C, mode="fp64", seed=spec["seed"],
                         stream_id=spec["stream_id"], radius0=radius0, max_steps=spec["max_steps"])


def _follow_oracle(specs, C, steps):
    """Step the batch and every instance's oracle search side by side: each
    candidate's FP64 mu within 1e-12, then selection, acceptance, radius and
    step while no near tie; returns the instances stopped at a near tie."""
    b = lib.Batch(specs, candidates=C, radius0=0.1).init()
    mu = b.query()[0]
    states = []
    for k, sp in enumerate(specs):
        p = _oracle_params(sp, C)
        st = oracle.haar_init(p)
        assert abs(mu[k] - st.mu) <= 1e-12
        states.append((p, st))
    stopped = set()
    for t in range(steps):
        b.step(1, report=True)
        rep_mu = b.rep_mu.cpu().numpy().reshape(len(specs), C)
        rep_best = b.rep_best.cpu().numpy()
        mu, radius, step, flags, done = b.query()
        for k, (p, st) in enumerate(states):
            if k in stopped:
                continue
            new, rep = oracle.step(p, st)
            assert np.max(np.abs(rep_mu[k] - rep.cand_mu)) <= 1e-12, f"instance {k} step {t}"
            if rep.near_tie or flags[k] & lib.FLAG_NEAR_TIE:
                stopped.add(k)
                continue
            assert rep_best[k] == rep.best and bool(flags[k] & lib.FLAG_ACCEPTED) == rep.accepted
            assert radius[k] == new.radius and step[k] == new.t and abs(mu[k] - new.mu) <= 1e-12
            states[k] = (p, new)
    return stopped


def test_batch_large_d_matches_oracle():
    """d = 9..16 (the reals fill the whole 32-wide screen step; N up to d^2):
    every candidate's exact mu through the split screen and its recheck."""
    specs = _specs(10, seed=13, d_lo=9, d_hi=16)
    stopped = _follow_oracle(specs, 16, 5)
    assert len(stopped) < len(specs)


def test_batch_long_run_on_small_instances_matches_oracle():
    """300 steps at d = 3, 4 (N up to d^2): the search evens out the largest
    pairs (6 to 13 pairs of each final frame lie within twice the screen's
    bound of its maximum), so the recheck re-evaluates several pairs per
    candidate; every candidate's exact mu still matches."""
    specs = [{"n": n, "d": d, "seed": 7, "stream_id": 500 + k, "max_steps": 10 ** 6, "waves_per_item": 0}
             for k, (d, n) in enumerate([(3, 9), (3, 7), (4, 16), (4, 12)])]
    stopped = _follow_oracle(specs, 16, 300)
    assert len(stopped) < len(specs)


def test_batch_edge_sizes_match_oracle():
    """d = 1 (every pair has |G| = 1, so every pair is rechecked) and d = 2,
    N = d + 1, and the largest instance (d = 16, N = 256): every candidate's
    exact mu through the split screen, its zero padding and its recheck."""
    sizes = [(1, 2), (1, 7), (2, 3), (2, 5), (3, 4), (16, 17), (16, 256)]
    specs = [{"n": n, "d": d, "seed": 3, "stream_id": 700 + k, "max_steps": 1000, "waves_per_item": 0}
             for k, (d, n) in enumerate(sizes)]
    _follow_oracle(specs, 16, 4)


def test_batch_matches_oracle_per_instance():
    C = 16
    specs = _specs(20, seed=3, d_hi=8)
    b = lib.Batch(specs, candidates=C, radius0=0.1).init()
    mu, radius, step, flags, done = b.query()
    states = []
    for k, sp in enumerate(specs):
        p = _oracle_params(sp, C)
        st = oracle.haar_init(p)
        assert np.max(np.abs(b.frame(k) - st.frame)) <= 1e-14
        assert abs(mu[k] - st.mu) <= 1e-12
        states.append((p, st))
    stopped = set()
    for t in range(8):
        b.step(1, report=True)
        rep_mu = b.rep_mu.cpu().numpy().reshape(len(specs), C)
        rep_best = b.rep_best.cpu().numpy()
        mu, radius, step, flags, done = b.query()
        for k, (p, st) in enumerate(states):
            if k in stopped:
                continue
            new, rep = oracle.step(p, st)
            assert np.max(np.abs(rep_mu[k] - rep.cand_mu)) <= 1e-12, f"instance {k} step {t}"
            if rep.near_tie or flags[k] & lib.FLAG_NEAR_TIE:
                stopped.add(k)
                continue
            assert rep_best[k] == rep.best
            assert bool(flags[k] & lib.FLAG_ACCEPTED) == rep.accepted
            assert radius[k] == new.radius and step[k] == new.t
            assert abs(mu[k] - new.mu) <= 1e-12
            states[k] = (p, new)
    assert len(stopped) < len(specs)
    for k, (p, st) in enumerate(states):
        if k not in stopped:
            assert np.max(np.abs(b.frame(k) - st.frame)) <= 1e-13


def _final(b, steps):
    b.step(steps)
    mu, radius, step, flags, _ = b.query()
    frames = [b.frame(k) for k in range(b.count)]
    return mu, radius, step, frames


def test_batch_result_independent_of_mix_and_tile():
    C, steps = 16, 12
    specs = _specs(16, seed=5, d_hi=16)
    full = _final(lib.Batch(specs, candidates=C).init(), steps)
    for k in (0, 5, 11):
        alone = _final(lib.Batch([specs[k]], candidates=C).init(), steps)
        assert alone[0][0] == full[0][k] and alone[1][0] == full[1][k] and alone[2][0] == full[2][k]
        assert np.array_equal(alone[3][0], full[3][k])
    for wpi in (1, 2, 4):
        ok = [dict(s, waves_per_item=wpi) for s in specs
              if s["n"] * autotune.ldk(s["d"]) * (4 // wpi) <= autotune.LDS_WORDS]
        idx = [k for k, s in enumerate(specs) if s["n"] * autotune.ldk(s["d"]) * (4 // wpi) <= autotune.LDS_WORDS]
        res = _final(lib.Batch(ok, candidates=C).init(), steps)
        for j, k in enumerate(idx):
            assert res[0][j] == full[0][k] and res[1][j] == full[1][k]
            assert np.array_equal(res[3][j], full[3][k])


def test_batch_graph_run_until_done_equals_launches():
    C = 8
    specs = _specs(12, seed=9, d_hi=6, max_steps=25)
    a = lib.Batch(specs, candidates=C).init()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        assert a.run(chunk=4, max_chunks=100, stream=s)
    s.synchronize()
    ma, ra, sa, fa, da = a.query()
    assert da == len(specs) and np.all(sa == 25) and np.all(fa & lib.FLAG_DONE)
    b = lib.Batch(specs, candidates=C).init()
    b.step(30)   # extra launches are no-ops once every instance is done
    mb, rb, sb, fb, db = b.query()
    assert np.array_equal(ma, mb) and np.array_equal(ra, rb) and np.array_equal(sa, sb)
    for k in range(len(specs)):
        assert np.array_equal(a.frame(k), b.frame(k))


def test_batch_target_stops_instance():
    specs = [{"n": 6, "d": 3, "seed": 1, "stream_id": 0, "target_mu": 0.99, "max_steps": 500},
             {"n": 20, "d": 4, "seed": 1, "stream_id": 1, "max_steps": 3}]
    b = lib.Batch(specs, candidates=8).init()
    b.step(10)
    mu, radius, step, flags, done = b.query()
    assert done == 2 and mu[0] <= 0.99 and step[1] == 3


def test_batch_full_workload_sampled():
    """512 instances, d in {3..16}, N in [d+1, d^2], 64 candidates: a few steps,
    sampled instances checked against the oracle."""
    C = 64
    specs = [{"n": n, "d": d, "seed": 0, "stream_id": k, "max_steps": 10 ** 6}
             for k, (d, n) in enumerate(inputs.batched_instances(512, seed=0))]
    b = lib.Batch(specs, candidates=C, radius0=0.1).init()
    b.step(3)
    mu, radius, step, flags, done = b.query()
    assert np.all(step == 3)
    rng = np.random.default_rng(1)
    for k in rng.choice(512, 6, replace=False):
        p = _oracle_params(specs[k], C)
        st = oracle.haar_init(p)
        near = False
        for _ in range(3):
            st, rep = oracle.step(p, st)
            near |= rep.near_tie
        if not near:
            assert abs(mu[k] - st.mu) <= 1e-12 and radius[k] == st.radius
