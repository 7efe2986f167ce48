"""Seeded synthetic inputs for the compressive light-sheet reconstruction.

The paper evaluates on a private synthetic zebrafish-heart volume (Sec. IV-A)
that is not available; these generators stand in for it with volumes of
Gaussian "nuclei" blobs, i.i.d. Bernoulli(1/2) DMD masks and a simulated coded
camera frame.

This module produces data only.  It is shared by the FP64 oracle tests and the
GPU tests so that both sides see bit-identical inputs, and it contains no step
of the reconstruction method.  The acquisition simulation (masked slices summed
on the camera, Sec. III-A, plus read/photon noise) is evaluated once here in
float64 and rounded to float32; neither the oracle nor the library uses it as
its operator.

Every draw comes from ``numpy.random.default_rng([20251103, config, snapshot])``
in this fixed order: blob centres/sizes/amplitudes, background, masks, noise.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 20251103


@dataclass
class Problem:
    """One coded snapshot and the settings used to reconstruct it."""

    gt: np.ndarray  # float32 [N*R][H][W] ground-truth volume in [0, 1]
    masks: np.ndarray  # uint8 [R][H][W], values {0, 1}
    y: np.ndarray  # float32 [N][H][W] coded frames
    params: dict = field(default_factory=dict)
    config: int = 0
    snapshot: int = 0

    @property
    def shape(self):
        nr, h, w = self.gt.shape
        return nr, h, w


# Reconstruction settings per workload.  lam is the TV weight, rho the ADMM
# penalty, gamma the z-smoothness weight; tv_inner/tv_tau drive the dual
# projection; iters is the fixed ADMM iteration count.
CONFIGS = {
    1: dict(H=256, W=256, B=8, n_blobs=40, background=False, noise=("gauss", 0.01),
            params=dict(denoiser="tv", lam=0.05, rho=1.0, gamma=0.0, iters=50,
                        tv_inner=10, tv_tau=0.125, zbc="periodic")),
    2: dict(H=512, W=512, B=16, n_blobs=300, background=True, noise=("poisson_gauss", 200.0, 0.01),
            params=dict(denoiser="tv", lam=0.05, rho=1.0, gamma=0.1, iters=100,
                        tv_inner=10, tv_tau=0.125, zbc="periodic")),
    3: dict(H=None, W=None, B=None, n_blobs=40, background=False, noise=("gauss", 0.01),
            params=dict(denoiser="tv", lam=0.05, rho=1.0, gamma=0.1, iters=100,
                        tv_inner=10, tv_tau=0.125, zbc="periodic")),
    4: dict(H=512, W=512, B=16, n_blobs=300, background=True, noise=("poisson_gauss", 200.0, 0.01),
            params=dict(denoiser="tv", lam=0.05, rho=1.0, gamma=0.1, iters=30,
                        tv_inner=10, tv_tau=0.125, zbc="periodic", ckpt_every=5)),
    5: dict(H=1024, W=1024, B=16, n_blobs=40, background=False, noise=("gauss", 0.02),
            params=dict(denoiser="bm3d", lam=0.05, rho=1.0, gamma=0.1, iters=30,
                        tv_inner=10, tv_tau=0.125, zbc="periodic", bm3d_sigma=9.669 / 255.0)),
}

BATCH_SIZES = [(256, 256), (512, 512), (768, 512), (1024, 1024)]
BATCH_DEPTHS = [8, 16, 24]


def _gauss_1d(coord, centre, sigma):
    # exp(-(c - centre)^2 / (2 sigma^2)) for every blob (rows) and coordinate (cols)
    return np.exp(-((coord[None, :] - centre[:, None]) ** 2) / (2.0 * sigma[:, None] ** 2))


def blob_volume(rng, B, H, W, n_blobs):
    """Sum of 3D Gaussian blobs evaluated in float64 at integer voxel coordinates.

    Draw order: cz~U[0,B), cy~U[0,H), cx~U[0,W), sigma_xy~U[3,6], sigma_z~U[1,2],
    a~U[0.3,1], each a vector of length n_blobs.  The Gaussian is separable, so
    the sum is accumulated slice by slice as a product of 1D profiles.
    """
    cz = rng.uniform(0.0, B, n_blobs)
    cy = rng.uniform(0.0, H, n_blobs)
    cx = rng.uniform(0.0, W, n_blobs)
    sxy = rng.uniform(3.0, 6.0, n_blobs)
    sz = rng.uniform(1.0, 2.0, n_blobs)
    amp = rng.uniform(0.3, 1.0, n_blobs)
    gz = _gauss_1d(np.arange(B, dtype=np.float64), cz, sz)  # [nb][B]
    gy = _gauss_1d(np.arange(H, dtype=np.float64), cy, sxy)  # [nb][H]
    gx = _gauss_1d(np.arange(W, dtype=np.float64), cx, sxy)  # [nb][W]
    vol = np.empty((B, H, W), dtype=np.float64)
    for z in range(B):
        wz = amp * gz[:, z]
        vol[z] = (gy.T * wz[None, :]) @ gx
    return vol


def background(rng, B, H, W):
    """Slowly varying background: low-pass filtered U[0,1] noise, min-max scaled, x0.1."""
    from scipy.ndimage import gaussian_filter

    raw = rng.random((B, H, W))
    bg = gaussian_filter(raw, sigma=(2.0, 16.0, 16.0), mode="wrap")
    lo, hi = bg.min(), bg.max()
    bg = (bg - lo) / (hi - lo) if hi > lo else np.zeros_like(bg)
    return 0.1 * bg


def bernoulli_masks(rng, R, H, W):
    return (rng.random((R, H, W)) < 0.5).astype(np.uint8)


def simulate_frames(gt64, masks, N, R):
    """Camera frames of the DMD-coded acquisition (Sec. III-A), float64, noise-free."""
    H, W = gt64.shape[1:]
    frames = np.zeros((N, H, W), dtype=np.float64)
    m = masks.astype(np.float64)
    for j in range(N):
        for r in range(R):
            frames[j] += m[r] * gt64[j * R + r]
    return frames


def add_noise(rng, y0, noise):
    kind = noise[0]
    if kind == "none":
        return y0.copy()
    if kind == "gauss":
        return y0 + rng.normal(0.0, noise[1], y0.shape)
    if kind == "poisson_gauss":
        scale, read = noise[1], noise[2]
        return rng.poisson(scale * np.maximum(y0, 0.0)) / scale + rng.normal(0.0, read, y0.shape)
    raise ValueError(f"unknown noise model {kind!r}")


def make_problem(H, W, R, N=1, n_blobs=40, bg=False, noise=("gauss", 0.01), seed=(0,),
                 params=None, config=0, snapshot=0, mask_p=0.5):
    """Generic generator; ``seed`` is appended to the base seed."""
    rng = np.random.default_rng([SEED_BASE, *seed])
    gt = blob_volume(rng, N * R, H, W, n_blobs)
    if bg:
        gt = gt + background(rng, N * R, H, W)
    if mask_p == 0.5:
        masks = bernoulli_masks(rng, R, H, W)
    else:
        masks = (rng.random((R, H, W)) < mask_p).astype(np.uint8)
    gt = np.clip(gt, 0.0, 1.0)
    gt32 = gt.astype(np.float32)
    y0 = simulate_frames(gt32.astype(np.float64), masks, N, R)
    y = add_noise(rng, y0, noise).astype(np.float32)
    return Problem(gt=gt32, masks=masks, y=y, params=dict(params or {}), config=config,
                   snapshot=snapshot)


def make(config, snapshot=0, **override):
    """Workload ``config`` (1..5); config 3 uses :func:`batch_shapes` for its sizes."""
    cfg = CONFIGS[config]
    H, W, B = cfg["H"], cfg["W"], cfg["B"]
    if config == 3:
        H, W, B = batch_shapes()[snapshot]
    H = override.pop("H", H)
    W = override.pop("W", W)
    B = override.pop("B", B)
    params = dict(cfg["params"])
    params.update(override.pop("params", {}))
    n_blobs = override.pop("n_blobs", cfg["n_blobs"])
    if override:
        raise TypeError(f"unknown overrides {sorted(override)}")
    return make_problem(H, W, B, 1, n_blobs, cfg["background"], cfg["noise"],
                        seed=(config, snapshot), params=params, config=config,
                        snapshot=snapshot)


def batch_shapes(n=64):
    """(H, W, R) of the batched workload's snapshots, drawn from rng([20251103, 3])."""
    rng = np.random.default_rng([SEED_BASE, 3])
    sizes = rng.integers(0, len(BATCH_SIZES), n)
    depths = rng.integers(0, len(BATCH_DEPTHS), n)
    return [(*BATCH_SIZES[s], BATCH_DEPTHS[b]) for s, b in zip(sizes, depths)]


def random_state(shape, seed, scale=0.1):
    """Seeded FP32 (u, d) pair for single-iteration tests."""
    rng = np.random.default_rng([SEED_BASE, 99, *seed])
    u = (rng.random(shape) * 1.0).astype(np.float32)
    d = (rng.normal(0.0, scale, shape)).astype(np.float32)
    return u, d
