"""Pins for the oracle's BM3D (CPU only): the transforms against their
definitions and an independent library DCT; block matching against brute
force and its tie-break rule; limiting cases of the two stages."""
import numpy as np
import pytest
from scipy.fft import dct

from oracle import bm3d as B


def test_dct_matches_library_and_is_orthonormal():
    C = B.dct_matrix()
    np.testing.assert_allclose(C @ C.T, np.eye(8), atol=1e-14)
    x = np.random.default_rng([61]).normal(size=8)
    np.testing.assert_allclose(C @ x, dct(x, type=2, norm="ortho"), atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
def test_haar_orthonormal_with_dc_row(n):
    Hm = B.haar_matrix(n)
    np.testing.assert_allclose(Hm @ Hm.T, np.eye(n), atol=1e-14)
    np.testing.assert_allclose(Hm[0], np.full(n, 1 / np.sqrt(n)), atol=1e-15)
    if n == 2:
        np.testing.assert_allclose(Hm, np.array([[1, 1], [1, -1]]) / np.sqrt(2), atol=1e-15)


def test_3d_transform_perfect_reconstruction():
    g = np.random.default_rng([62]).normal(size=(8, 8, 8))
    C = B.dct_matrix()
    np.testing.assert_allclose(B.itransform3d(B.transform3d(g, C), C), g, atol=1e-13)
    # Parseval
    assert abs(np.sum(B.transform3d(g, C) ** 2) - np.sum(g ** 2)) < 1e-11


def test_reference_grid_covers_image():
    assert B.ref_positions(8) == [0]
    assert B.ref_positions(20) == [0, 3, 6, 9, 12]
    assert B.ref_positions(21) == [0, 3, 6, 9, 12, 13]


def test_matching_equals_brute_force():
    rng = np.random.default_rng([63])
    img = rng.random((30, 27))
    for (ry, rx) in [(0, 0), (9, 12), (22, 19), (13, 0)]:
        grp = B.match(img, ry, rx, tau=0.2)
        H, W = img.shape
        cands = []
        for y in range(H - 7):
            for x in range(W - 7):
                if abs(y - ry) <= 19 and abs(x - rx) <= 19 and (y, x) != (ry, rx):
                    d = np.mean((img[ry:ry + 8, rx:rx + 8] - img[y:y + 8, x:x + 8]) ** 2)
                    if d <= 0.2:
                        cands.append((d, y * W + x, (y, x)))
        cands.sort()
        ref = [(ry, rx)] + [c[2] for c in cands[:15]]
        n = 1
        while 2 * n <= len(ref):
            n *= 2
        assert grp == ref[:n]


def test_tie_break_by_raster_index():
    img = np.full((20, 20), 0.3)
    grp = B.match(img, 6, 6, tau=B.TAU_HT)
    # all distances are 0: the reference, then candidates in raster order
    ys = range(0, 13)
    expect = [(6, 6)] + [(y, x) for y in ys for x in range(0, 13) if (y, x) != (6, 6)][:15]
    assert grp == expect


def test_limits_small_sigma_identity_and_constant():
    rng = np.random.default_rng([64])
    img = rng.random((24, 26))
    out = B.bm3d_slice(img, 1e-9)
    np.testing.assert_allclose(out, img, atol=1e-10)
    # a constant image stays constant: the hard-threshold stage returns it exactly, the Wiener
    # stage shrinks its DC coefficient B by B^2/(B^2 + sigma^2) (B = 8 c sqrt(n) for n blocks)
    c = np.full((16, 19), 0.42)
    out, basic = B.bm3d_slice(c, 0.05, return_basic=True)
    np.testing.assert_allclose(basic, c, atol=1e-14)
    assert np.ptp(out) < 1e-12
    n = 16
    dc = 8 * 0.42 * np.sqrt(n)
    assert abs(out[0, 0] - 0.42 * dc * dc / (dc * dc + 0.05 ** 2)) < 1e-12


def test_denoises_a_smooth_image():
    y, x = np.mgrid[0:40, 0:40]
    clean = 0.5 + 0.3 * np.sin(x / 6.0) * np.cos(y / 7.0)
    noisy = clean + np.random.default_rng([65]).normal(0, 0.05, clean.shape)
    out = B.bm3d_slice(noisy, 0.05)
    assert np.linalg.norm(out - clean) < 0.6 * np.linalg.norm(noisy - clean)
