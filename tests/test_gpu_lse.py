"""GPU parity: trstmi_lse (the smooth maximum of section IV) against the oracle."""

import math

import numpy as np
import pytest

import frames
import inputs
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
lib = pytest.importorskip("paper_2207_06374_amd")


def _gpu(F, delta, squared=True):
    d, n = F.shape
    out = lib.lse(lib.frame_to_device(F), n, d, delta, squared)
    s, f = out.cpu().numpy().tolist()
    return s, f


def _tol(n_vec, delta):
    # FP64 x differs from the oracle's by a few ulp (moving each exp by about
    # 1e-16 / delta relative, i.e. 1e-16 absolute in F); the GPU adds the n
    # terms in blocks (relative error at most n 2^-53 of the sum)
    n = n_vec * (n_vec - 1) // 2
    return 1e-13 + delta * n * 2.0 ** -52


SHAPES = [(2, 1), (3, 2), (16, 4), (65, 3), (100, 7), (129, 5), (200, 16), (257, 33), (300, 64), (70, 130)]


@pytest.mark.parametrize("n,d", SHAPES)
@pytest.mark.parametrize("delta", [0.1, 1e-2, 1e-3])
def test_lse_matches_oracle(n, d, delta):
    F = inputs.random_frame(n, d, seed=n * 31 + d)
    for squared in (True, False):
        s_ref, f_ref = oracle.smooth_max(F, delta, squared)
        s, f = _gpu(F, delta, squared)
        print(f"n={n} d={d} delta={delta} squared={squared} ref=({s_ref!r}, {f_ref!r}) got=({s!r}, {f!r})",
              flush=True)
        assert abs(s - s_ref) <= 1e-14
        assert abs(f - f_ref) <= _tol(n, delta)
        npairs = n * (n - 1) // 2
        assert s <= f <= s + delta * math.log(npairs) * (1 + 1e-12) + 1e-15


def test_lse_closed_forms():
    F = np.array([[1, 0, 1], [0, 1, 1]], dtype=complex)
    s, f = _gpu(F, 0.05)
    assert abs(s - 0.5) <= 1e-15
    assert abs(f - (0.5 + 0.05 * math.log(2 + math.exp(-10.0)))) <= 1e-14
    F = frames.sic_numeric(4)
    s, f = _gpu(F, 0.01)
    assert abs(s - 0.2) <= 1e-13 and abs(f - (0.2 + 0.01 * math.log(120))) <= 1e-11
    build, mu = frames.KNOWN["hesse"]
    s, f = _gpu(build(), 1e-3)
    assert abs(s - mu * mu) <= 1e-14 and abs(f - (mu * mu + 1e-3 * math.log(36))) <= 1e-12


def test_lse_invalid_column_and_repeatability():
    F = inputs.random_frame(50, 4, seed=3)
    F[:, 7] = 0
    assert _gpu(F, 0.1) == (math.inf, math.inf)
    F = inputs.random_frame(300, 16, seed=5)
    dev = lib.frame_to_device(F)
    a = lib.lse(dev, 300, 16, 1e-3).cpu().numpy()
    b = lib.lse(dev, 300, 16, 1e-3).cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_lse_full_size():
    """The throughput workload's shape: a 4096 x 64 Haar frame."""
    p = oracle.Params(n=4096, d=64, seed=0)
    F = oracle.haar_init(p).frame
    for delta in (1e-2, 1e-3):
        s_ref, f_ref = oracle.smooth_max(F, delta)
        s, f = _gpu(F, delta)
        assert abs(s - s_ref) <= 1e-14
        assert abs(f - f_ref) <= _tol(4096, delta)


def _gpu_grad(F, delta):
    d, n = F.shape
    out, g = lib.lse_grad(lib.frame_to_device(F), n, d, delta)
    return out.cpu().numpy().tolist(), lib.frame_from_device(g, n, d)


# every output row-block count MB = ceil(2d / 16) of the kernel (d = 8 | 9,
# 16 | 17, 32 | 33, 40 | 41, 48, 56, 64), ragged tiles
GRAD_SHAPES = [(2, 1), (3, 2), (16, 4), (65, 3), (100, 7), (150, 8), (90, 9), (129, 5), (200, 16), (130, 20),
               (77, 32), (257, 33), (140, 45), (70, 56), (300, 64)]


@pytest.mark.parametrize("n,d", GRAD_SHAPES)
@pytest.mark.parametrize("delta", [0.1, 1e-2, 1e-3])
def test_lse_grad_matches_oracle(n, d, delta):
    rng = np.random.default_rng(n + d)
    F = inputs.random_frame(n, d, seed=n * 7 + d) * (0.5 + rng.random(n))[None, :]   # unnormalised columns
    (s, f), g = _gpu_grad(F, delta)
    s_ref, f_ref = oracle.smooth_max(F, delta)
    g_ref = oracle.smooth_max_grad(F, delta)
    err = float(np.max(np.abs(g - g_ref)))
    print(f"n={n} d={d} delta={delta} |g|max={float(np.max(np.abs(g_ref)))!r} err={err!r}", flush=True)
    assert abs(s - s_ref) <= 1e-14 and abs(f - f_ref) <= _tol(n, delta)
    assert err <= 2e-11 * max(1.0, float(np.max(np.abs(g_ref))))
    # no radial component (F is invariant to column scale)
    Phi, _ = oracle.normalize_columns(F)
    assert float(np.max(np.abs(np.sum((Phi.conj() * g).real, axis=0)))) <= 1e-12


def test_lse_grad_invalid_repeatable_and_full_size():
    F = inputs.random_frame(70, 5, seed=1)
    F[:, 3] = np.nan
    (s, f), g = _gpu_grad(F, 0.1)
    assert s == math.inf and f == math.inf and np.all(np.isnan(g))
    F = inputs.random_frame(300, 32, seed=2)
    dev = lib.frame_to_device(F)
    _, g1 = lib.lse_grad(dev, 300, 32, 1e-2)
    _, g2 = lib.lse_grad(dev, 300, 32, 1e-2)
    assert np.array_equal(g1.cpu().numpy().view(np.uint64), g2.cpu().numpy().view(np.uint64))
    p = oracle.Params(n=4096, d=64, seed=0)
    F = oracle.haar_init(p).frame
    (s, f), g = _gpu_grad(F, 1e-3)
    g_ref = oracle.smooth_max_grad(F, 1e-3)
    assert float(np.max(np.abs(g - g_ref))) <= 2e-11 * max(1.0, float(np.max(np.abs(g_ref))))


def test_lse_grad_many_row_runs():
    """A frame whose row tiles are split into many runs per column block (47
    tiles a side), against the oracle."""
    n, d, delta = 3000, 4, 1e-2
    F = inputs.random_frame(n, d, seed=31)
    (s, f), g = _gpu_grad(F, delta)
    s_ref, f_ref = oracle.smooth_max(F, delta)
    g_ref = oracle.smooth_max_grad(F, delta)
    assert abs(s - s_ref) <= 1e-14 and abs(f - f_ref) <= _tol(n, delta)
    assert float(np.max(np.abs(g - g_ref))) <= 2e-11 * max(1.0, float(np.max(np.abs(g_ref))))
