"""Pins for the oracle's random draws (CPU only)."""

import math

import numpy as np
import pytest
from scipy import stats

import oracle
from conftest import golden_path


def _kat_rows():
    rows = []
    for line in open(golden_path("philox4x32_10_kat.txt")):
        if line.strip() and not line.startswith("#"):
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat_rows()
    assert len(rows) == 3
    for ctr, key, out in rows:
        got = oracle.philox4x32_10(np.array(ctr), np.array(key))
        assert [int(x) for x in got] == out


def test_philox_vectorised_equals_scalar():
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2 ** 32, size=(50, 4), dtype=np.uint64)
    key = np.array([123456789, 987654321], dtype=np.uint64)
    batch = oracle.philox4x32_10(ctr, key)
    for i in range(50):
        assert np.array_equal(batch[i], oracle.philox4x32_10(ctr[i], key))


def test_uniform_range_and_extremes():
    u = oracle.uniforms_from_words(np.array([0, 2 ** 32 - 1], dtype=np.uint64))
    assert u[0] == 2.0 ** -33
    assert u[1] == 1.0 - 2.0 ** -33
    assert np.all((u > 0) & (u < 1))


def test_box_muller_is_standard_normal():
    rng = np.random.default_rng(0)
    u0 = (rng.integers(0, 2 ** 32, 400000) + 0.5) * 2.0 ** -32
    u1 = (rng.integers(0, 2 ** 32, 400000) + 0.5) * 2.0 ** -32
    g0, g1 = oracle.box_muller(u0, u1)
    for g in (g0, g1):
        assert stats.kstest(g, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(g0, g1)[0, 1]) < 0.01


def test_frame_entries_complex_normal():
    Z = oracle.complex_gaussian_frame(2048, 7, seed=11, stream_id=2, cand=3, t=5, tag=oracle.TAG_PERTURB)
    assert Z.shape == (7, 2048)
    z = Z.ravel()
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 0.02          # E|z|^2 = 1
    assert abs(np.mean(z * z)) < 0.02                         # circular: E z^2 = 0
    assert abs(np.mean(z)) < 0.03
    for part in (z.real, z.imag):
        assert stats.kstest(part * math.sqrt(2), "norm").pvalue > 1e-4
    # entries 2q and 2q+1 of a column (same block) and neighbouring columns are uncorrelated
    assert abs(np.corrcoef(Z[0].real, Z[1].real)[0, 1]) < 0.08
    assert abs(np.corrcoef(Z[0, :-1].real, Z[0, 1:].real)[0, 1]) < 0.08


def test_streams_are_distinct():
    base = dict(n=64, d=4, seed=1, stream_id=0, cand=0, t=0, tag=0)
    ref = oracle.complex_gaussian_frame(**base)
    for k, v in [("seed", 2), ("stream_id", 1), ("cand", 1), ("t", 1), ("tag", 1)]:
        other = oracle.complex_gaussian_frame(**{**base, k: v})
        assert abs(np.corrcoef(ref.real.ravel(), other.real.ravel())[0, 1]) < 0.3
        assert not np.any(ref == other)


def test_counter_layout_odd_d():
    """For odd d each column owns ceil(d/2) blocks: the first d rows of a
    (d+1)-row draw are the d-row draw."""
    a = oracle.complex_gaussian_frame(10, 5, 1, 0, 0, 0, 0)
    b = oracle.complex_gaussian_frame(10, 6, 1, 0, 0, 0, 0)
    assert np.array_equal(a, b[:5])
    # batched candidates equal single draws
    many = oracle.complex_gaussian_frame(10, 5, 1, 0, np.arange(3), 4, 0)
    assert np.array_equal(many[2], oracle.complex_gaussian_frame(10, 5, 1, 0, 2, 4, 0))


@pytest.mark.parametrize("d", [2, 4, 9])
def test_haar_columns_beta_law(d):
    """For independent uniformly random unit vectors in C^d, |<x,y>|^2 ~ Beta(1, d-1)."""
    p = oracle.Params(n=3000, d=d, seed=5)
    st = oracle.haar_init(p)
    F = st.frame
    assert np.allclose(np.linalg.norm(F, axis=0), 1.0, atol=1e-14)
    x = np.abs(np.sum(np.conj(F[:, 0::2]) * F[:, 1::2], axis=0)) ** 2
    assert stats.kstest(x, stats.beta(1, d - 1).cdf).pvalue > 1e-4


def test_rounding_bf16_against_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x32 = (rng.standard_normal(20000) * 10.0 ** rng.uniform(-6, 0, 20000)).astype(np.float32)
    ours = oracle.round_to_bf16(x32.astype(np.float64))
    theirs = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ours, theirs)


def test_rounding_bf16_ties_to_even():
    one = 1.0
    assert oracle.round_to_bf16(np.array([one + 2 ** -8]))[0] == 1.0
    assert oracle.round_to_bf16(np.array([one + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6
    assert oracle.round_to_bf16(np.array([-(one + 2 ** -8 + 2 ** -20)]))[0] == -(1.0 + 2 ** -7)
    assert oracle.round_to_bf16(np.array([0.0]))[0] == 0.0
    # subnormal range: spacing 2^-133
    assert oracle.round_to_bf16(np.array([3 * 2.0 ** -134]))[0] == 2 * 2.0 ** -133


def test_rounding_fp32():
    x = np.array([1.0 + 2 ** -30, 0.1])
    r = oracle.round_to_fp32(x)
    assert r[0] == 1.0 and r[1] == float(np.float32(0.1))
