"""Reconstruction-quality metrics of the experiments (oracle), and the
relative-change stopping test.

Sec. IV: PSNR(I^, I) = 10 log10(m n V^2 / ||I^ - I||^2), V the peak intensity;
in 3D all voxels form one array.  SSIM: local statistics under an 11 x 11
Gaussian window of standard deviation 1.5 (11 x 11 x 11 in 3D),
c1 = (0.01 L)^2, c2 = (0.03 L)^2 with L = 1, averaged over the window
positions.  Readings: the window is normalised to sum 1; local variances and
covariance are the window-weighted moments about the local means; positions
are those where the whole window lies inside the data ("valid"), so the 3D
index needs at least 11 slices.

Stopping (Sec. IV-B names a relative tolerance without defining it):
rel = ||x^{k+1} - x^k|| / ||x^k||.
"""
import numpy as np

WIN = 11
SIGMA = 1.5


def gaussian_window():
    t = np.arange(WIN) - (WIN - 1) / 2.0
    g = np.exp(-(t * t) / (2.0 * SIGMA * SIGMA))
    return g / g.sum()


def psnr(est, ref, peak=1.0):
    est = np.asarray(est, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.sum((est - ref) ** 2)
    return 10.0 * np.log10(est.size * peak * peak / err)


def _window_sums(a, axes):
    """Window-weighted sum over the valid positions along each of `axes`."""
    g = gaussian_window()
    out = np.asarray(a, dtype=np.float64)
    for ax in axes:
        n = out.shape[ax]
        if n < WIN:
            raise ValueError("each windowed axis needs at least 11 samples")
        moved = np.moveaxis(out, ax, -1)
        acc = np.zeros(moved.shape[:-1] + (n - WIN + 1,))
        for k in range(WIN):
            acc += g[k] * moved[..., k:k + n - WIN + 1]
        out = np.moveaxis(acc, -1, ax)
    return out


def _ssim_map(x, y, axes, L):
    c1 = (0.01 * L) ** 2
    c2 = (0.03 * L) ** 2
    mx = _window_sums(x, axes)
    my = _window_sums(y, axes)
    sxx = _window_sums(x * x, axes) - mx * mx
    syy = _window_sums(y * y, axes) - my * my
    sxy = _window_sums(x * y, axes) - mx * my
    return ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))


def ssim2d(est, ref, L=1.0):
    """Mean 2D SSIM over every valid window position of every slice of [..., H, W] arrays."""
    x = np.asarray(est, dtype=np.float64)
    y = np.asarray(ref, dtype=np.float64)
    return float(np.mean(_ssim_map(x, y, (-1, -2), L)))


def ssim3d(est, ref, L=1.0):
    """Mean 3D SSIM (11 x 11 x 11 Gaussian window) over the valid positions of [D, H, W] volumes."""
    x = np.asarray(est, dtype=np.float64)
    y = np.asarray(ref, dtype=np.float64)
    return float(np.mean(_ssim_map(x, y, (-1, -2, -3), L)))


def rel_change(x_new, x_old):
    x_new = np.asarray(x_new, dtype=np.float64)
    x_old = np.asarray(x_old, dtype=np.float64)
    return float(np.linalg.norm(x_new - x_old) / np.linalg.norm(x_old))
