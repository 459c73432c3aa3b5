"""GPU parity: trstmi_coherence and the random start / candidates against the oracle."""

import math

import numpy as np
import pytest

import frames
import inputs
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lib = pytest.importorskip("paper_2207_06374_amd")


def _gpu_mu(F, mode):
    d, n = F.shape
    dev = lib.frame_to_device(F)
    return float(lib.coherence(dev, n, d, mode).item())


SHAPES = [(2, 1), (3, 2), (16, 4), (65, 3), (100, 7), (129, 5), (200, 16), (257, 33), (300, 64), (64, 128),
          (130, 100), (1000, 32), (70, 200), (40, 300), (33, 512)]


@pytest.mark.parametrize("n,d", SHAPES)
def test_coherence_fp64_random(n, d):
    F = inputs.random_frame(n, d, seed=n * 1000 + d)
    ref = oracle.coherence(F)
    got = _gpu_mu(F, lib.MODE_FP64)
    print(f"n={n} d={d} ref={ref!r} got={got!r}", flush=True)
    assert abs(got - ref) <= 1e-12


@pytest.mark.parametrize("name", sorted(frames.KNOWN))
def test_coherence_fp64_known_frames(name):
    build, mu = frames.KNOWN[name]
    F = build()
    got = _gpu_mu(F, lib.MODE_FP64)
    assert abs(got - mu) <= 1e-12


def test_coherence_fp64_numeric_sic():
    F = frames.sic_numeric(4)
    assert abs(_gpu_mu(F, lib.MODE_FP64) - math.sqrt(0.2)) <= 1e-12


@pytest.mark.parametrize("n,d", SHAPES)
def test_coherence_fp32_random(n, d):
    F = inputs.random_frame(n, d, seed=7 + n + d)
    ref = oracle.coherence(F)
    got = _gpu_mu(F, lib.MODE_FP32)
    assert abs(got - ref) <= 2e-6


@pytest.mark.parametrize("n,d", SHAPES)
def test_coherence_bf16_screen_within_bound(n, d):
    F = inputs.random_frame(n, d, seed=11 + n + d)
    exact = oracle.coherence(F)
    Fn, _ = oracle.normalize_columns(F)
    emul = oracle.evaluate_candidates(Fn[None], np.array([True]), "bf16")[0]
    got = _gpu_mu(F, lib.MODE_BF16_SCREEN)
    assert abs(got - exact) <= oracle.screen_error_bound(d)
    # same bf16 inputs: only the FP32 accumulation differs
    assert abs(got - emul) <= 2e-5


@pytest.mark.parametrize("mode", [lib.MODE_FP64, lib.MODE_FP32, lib.MODE_BF16_SCREEN])
def test_zero_and_nonfinite_column_give_inf(mode):
    F = inputs.random_frame(40, 5, seed=3)
    F[:, 17] = 0
    assert _gpu_mu(F, mode) == math.inf
    F = inputs.random_frame(40, 5, seed=3)
    F[2, 33] = np.inf
    assert _gpu_mu(F, mode) == math.inf


def test_coherence_full_size_haar():
    """Full-size 4096 x 64 frame (the throughput workload's shape)."""
    p = oracle.Params(n=4096, d=64, seed=0)
    F = oracle.haar_init(p).frame
    ref = oracle.coherence(F)
    assert abs(_gpu_mu(F, lib.MODE_FP64) - ref) <= 1e-12
    assert abs(_gpu_mu(F, lib.MODE_FP32) - ref) <= 2e-6
    got = _gpu_mu(F, lib.MODE_BF16_SCREEN)
    assert abs(got - ref) <= oracle.screen_error_bound(64)
    # same bf16 inputs as the oracle's emulation: only the FP32 accumulation differs
    Fn, _ = oracle.normalize_columns(F)
    emul = oracle.evaluate_candidates(Fn[None], np.array([True]), "bf16")[0]
    assert abs(got - emul) <= 2e-5


@pytest.mark.parametrize("n,d,seed,stream", [(16, 4, 0, 0), (33, 5, 7, 3), (1024, 32, 0, 0), (300, 64, 9, 1),
                                             (50, 1, 2, 0)])
def test_haar_start_parity(n, d, seed, stream):
    s = lib.Solver(n, d, seed=seed, stream_id=stream, mode="fp64")
    s.init_haar()
    F, mu, radius, t, flags = s.host_state()
    ref = oracle.haar_init(oracle.Params(n=n, d=d, seed=seed, stream_id=stream))
    assert np.max(np.abs(F - ref.frame)) <= 1e-14
    assert abs(mu - ref.mu) <= 1e-12
    assert radius == 0.1 and t == 0 and flags == 0


# every column split of the candidate kernel: d = 4 and 7 (partial), 16, 32,
# 64, 128 and 256 (full splits), 130 (wide partial)
@pytest.mark.parametrize("n,d,C,t", [(16, 4, 64, 0), (37, 7, 9, 5), (1024, 32, 4, 123), (70, 130, 3, 2),
                                     (90, 16, 5, 1), (200, 64, 3, 7), (129, 128, 2, 1), (40, 256, 2, 3)])
def test_candidates_parity(n, d, C, t):
    p = oracle.Params(n=n, d=d, candidates=C, seed=1, stream_id=2)
    st = oracle.haar_init(p)
    params = lib.default_params(n, d, candidates=C, seed=1, stream_id=2)
    frame = lib.frame_to_device(st.frame)
    radius = torch.tensor([0.05], dtype=torch.float64, device="cuda")
    out = lib.candidates(params, frame, radius, t, 0, C)
    got = out.cpu().numpy().reshape(C, n, d, 2)
    got = (got[..., 0] + 1j * got[..., 1]).transpose(0, 2, 1)
    Z = oracle.perturbations(p, t)
    ref, valid = oracle.make_candidates(st.frame, 0.05, d, Z)
    assert valid.all()
    assert np.max(np.abs(got - ref)) <= 1e-14


def test_candidates_explicit_z_and_invalid_column():
    n, d = 20, 3
    F = inputs.random_frame(n, d, 1)
    Fn, _ = oracle.normalize_columns(F)
    Z = inputs.random_perturbation(n, d, 2, seed=5)
    s = 0.3 / math.sqrt(d)
    Z[1][:, 4] = np.nan                                   # candidate 1, column 4: non-finite
    params = lib.default_params(n, d, candidates=2)
    zdev = torch.from_numpy(np.ascontiguousarray(np.transpose(Z, (0, 2, 1))).view(np.float64).ravel().copy()).cuda()
    out = lib.candidates(params, lib.frame_to_device(Fn), torch.tensor([0.3], dtype=torch.float64, device="cuda"),
                         0, 0, 2, explicit_z=zdev)
    got = out.cpu().numpy().reshape(2, n, d, 2)
    got = (got[..., 0] + 1j * got[..., 1]).transpose(0, 2, 1)
    ref, valid = oracle.make_candidates(Fn, 0.3, d, Z)
    assert valid[0] and not valid[1]
    assert np.max(np.abs(got[0] - ref[0])) <= 1e-15
    assert np.all(np.isnan(got[1][:, 4]))
    assert np.max(np.abs(np.delete(got[1], 4, axis=1) - np.delete(ref[1], 4, axis=1))) <= 1e-15


def test_round_bf16_matches_oracle_bitwise():
    """The rounding of the BF16 screen copies equals the oracle's direct
    round-to-nearest-even from FP64, bit for bit, including exact bfloat16
    midpoints, values within a float32 ulp of them (where rounding through
    float32 first would go wrong) and the subnormal ranges."""
    rng = np.random.default_rng(5)
    parts = [rng.standard_normal(200000) * np.exp2(rng.integers(-140, 40, 200000).astype(np.float64))]
    b = rng.standard_normal(50000).astype(np.float32)
    b = (b.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)            # bfloat16 values
    up = (b.view(np.uint32) + np.uint32(0x10000)).view(np.float32)              # next one away from 0
    m = (b.astype(np.float64) + up.astype(np.float64)) / 2                     # exact midpoints
    tiny = np.abs(m) * 2.0 ** -40
    parts += [m, m + tiny, m - tiny, np.nextafter(m, np.inf), np.nextafter(m, -np.inf)]
    parts.append(rng.standard_normal(20000) * 2.0 ** -130)
    parts.append(rng.standard_normal(20000) * 2.0 ** -145)
    parts.append(np.array([0.0, -0.0, 1.0, -1.0, 2.0 ** -126, 2.0 ** -133, 2.0 ** -134, 3 * 2.0 ** -135]))
    x = np.concatenate(parts)
    got = lib.round_bf16(torch.from_numpy(x).cuda()).cpu().numpy().view(np.uint16)
    ref = oracle.round_to_bf16(x)
    ref_bits = (ref.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    bad = np.flatnonzero(got != ref_bits)
    assert bad.size == 0, (x[bad[:5]], got[bad[:5]], ref_bits[bad[:5]])
    y = np.array([np.nan, np.inf, -np.inf])  # odd count
    g = lib.round_bf16(torch.from_numpy(y).cuda()).cpu().numpy().view(np.uint16)
    assert (g[0] & 0x7F80) == 0x7F80 and (g[0] & 0x7F) != 0
    assert g[1] == 0x7F80 and g[2] == 0xFF80


def _gpu_pair(F):
    d, n = F.shape
    mu, pair = lib.coherence_pair(lib.frame_to_device(F), n, d)
    return float(mu.item()), tuple(int(x) for x in pair.cpu().numpy())


@pytest.mark.parametrize("n,d", [(2, 1), (3, 2), (16, 4), (65, 3), (129, 5), (257, 33), (300, 64), (70, 200),
                                 (1000, 32)])
def test_coherence_pair_matches_oracle(n, d):
    """The pair's modulus is the coherence; on random frames the maximum is
    unique by a wide margin, so the pair is the oracle's."""
    F = inputs.random_frame(n, d, seed=n + 17 * d)
    mu, (j, k) = _gpu_pair(F)
    ref, rj, rk = oracle.coherence_pair(F)
    print(f"n={n} d={d} mu={mu!r} pair=({j},{k}) ref=({rj},{rk})", flush=True)
    assert abs(mu - ref) <= 1e-12 and 0 <= j < k < n
    Phi, _ = oracle.normalize_columns(F)
    assert abs(abs(np.vdot(Phi[:, j], Phi[:, k])) - ref) <= 1e-12
    G = np.abs(Phi.conj().T @ Phi)
    top = np.sort(G[np.triu_indices(n, 1)])[-2:]
    if top.size == 1 or top[1] - top[0] > 1e-12:
        assert (j, k) == (rj, rk)
    assert _gpu_mu(F, lib.MODE_FP64) == mu


def test_coherence_pair_ties_invalid_and_full_size():
    mu, pair = _gpu_pair(np.array([[1.0, 0.0, 1.0], [0.0, 1.0, 1.0]], dtype=complex))
    assert pair == (0, 2) and abs(mu - math.sqrt(0.5)) <= 2.3e-16
    for name in sorted(frames.KNOWN):
        build, ref = frames.KNOWN[name]
        F = build()
        mu, (j, k) = _gpu_pair(F)
        Phi, _ = oracle.normalize_columns(F)
        assert abs(mu - ref) <= 1e-12 and 0 <= j < k and abs(abs(np.vdot(Phi[:, j], Phi[:, k])) - ref) <= 1e-12
    F = inputs.random_frame(40, 5, seed=3)
    F[:, 17] = 0
    assert _gpu_pair(F) == (math.inf, (-1, -1))
    F = oracle.haar_init(oracle.Params(n=4096, d=64, seed=0)).frame
    mu, pair = _gpu_pair(F)
    ref, rj, rk = oracle.coherence_pair(F)
    assert abs(mu - ref) <= 1e-12 and pair == (rj, rk)
