"""Pins for the oracle's quality metrics (CPU only): closed forms for constant
images and offsets, identity, symmetry, and the windowed moments against a
brute-force sum at sampled positions."""
import numpy as np

from oracle import metrics as M


def test_window_normalised_and_symmetric():
    g = M.gaussian_window()
    assert abs(g.sum() - 1) < 1e-15
    np.testing.assert_allclose(g, g[::-1], atol=0)
    assert np.argmax(g) == 5


def test_psnr_closed_form():
    ref = np.random.default_rng([91]).random((4, 20, 30))
    est = ref + 0.01
    assert abs(M.psnr(est, ref) - 40.0) < 1e-9
    assert abs(M.psnr(est, ref, peak=2.0) - (40.0 + 20 * np.log10(2))) < 1e-9


def test_ssim_identity_symmetry_and_constants():
    rng = np.random.default_rng([92])
    x = rng.random((2, 30, 25))
    y = np.clip(x + rng.normal(0, 0.05, x.shape), 0, 1)
    assert abs(M.ssim2d(x, x) - 1.0) < 1e-12
    assert abs(M.ssim2d(x, y) - M.ssim2d(y, x)) < 1e-12
    assert M.ssim2d(x, y) < 1.0
    a, b = 0.3, 0.7
    c1 = 0.01 ** 2
    closed = (2 * a * b + c1) / (a * a + b * b + c1)
    assert abs(M.ssim2d(np.full((15, 16), a), np.full((15, 16), b)) - closed) < 1e-12
    v = rng.random((12, 14, 13))
    assert abs(M.ssim3d(v, v) - 1.0) < 1e-12
    assert abs(M.ssim3d(np.full((11, 12, 11), a), np.full((11, 12, 11), b)) - closed) < 1e-12


def test_windowed_moments_match_brute_force():
    rng = np.random.default_rng([93])
    x = rng.random((17, 19))
    g = M.gaussian_window()
    w2 = np.outer(g, g)
    mu = M._window_sums(x, (-1, -2))
    assert mu.shape == (7, 9)
    for (i, j) in [(0, 0), (3, 4), (6, 8)]:
        assert abs(mu[i, j] - np.sum(w2 * x[i:i + 11, j:j + 11])) < 1e-13


def test_rel_change():
    a = np.ones((3, 4))
    assert abs(M.rel_change(a * 1.01, a) - 0.01) < 1e-14
