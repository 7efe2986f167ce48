"""Plug-and-play ADMM for the coded light-sheet volume (oracle).

Objective (Sec. III-C, 1/2 on the data term as in the temporal model):

    1/2 sum_j ||b_j - sum_r phi_r v_{(j-1)R+r}||^2 + lambda sum_n psi(v_n)
        + (gamma/2) sum over adjacent z-pairs ||v_n - v_{n-1}||^2.

Splitting v = u with scaled dual d (Sec. III-B, eq. (ADMM)).  Two schedules:

* :func:`iterate` / :func:`solve` -- the temporal term is carried by the
  v-block, so the x-step is the per-pixel z-solve of :mod:`oracle.xstep`; the
  u-step denoises every slice of x + d independently at strength lambda/rho;
  then d <- d + x - u.  With gamma = 0 this is Algorithm 1 exactly.
* :func:`iterate_paper` / :func:`solve_paper` -- Algorithm 1 as printed: the
  v-step is eq. (v-update) (no gamma), and the u-step is one Gauss-Seidel sweep
  n = 1..NR of eq. (u-update): slice n denoises
  (rho (v_n + d_n) + gamma (u_{n-1} + u_{n+1})) / (rho + 2 gamma) at strength
  lambda / (rho + 2 gamma), using the newest neighbour values available.

Initialisation u = d = 0 unless a state is passed in; the x returned is the
last x-step result (Algorithm 1 returns v).
"""
from dataclasses import dataclass, replace

import numpy as np

from .denoise import denoise
from .laplacian import temporal_energy
from .operator import forward
from .tv import tv_value
from .xstep import xstep


@dataclass
class Params:
    lam: float = 0.05
    rho: float = 1.0
    gamma: float = 0.0
    iters: int = 50
    tv_inner: int = 10
    tv_tau: float = 0.125
    zbc: str = "periodic"
    denoiser: str = "tv"
    bm3d_sigma: float = 9.669 / 255.0

    @classmethod
    def from_dict(cls, d):
        keys = cls.__dataclass_fields__.keys()
        return cls(**{k: v for k, v in d.items() if k in keys})

    def with_(self, **kw):
        return replace(self, **kw)


def _zeros_state(b, masks):
    R = np.asarray(masks).shape[0]
    N, H, W = np.asarray(b).shape
    z = np.zeros((N * R, H, W), dtype=np.float64)
    return z, z.copy()


def iterate(b, masks, u, d, p):
    """One ADMM iteration with the temporal term in the x-step; returns (x, u, d)."""
    x = xstep(b, u, d, masks, p.rho, p.gamma, p.zbc)
    f = x + d
    u_new = denoise(f, p)
    d_new = f - u_new
    return x, u_new, d_new


def solve(b, masks, p, u=None, d=None, callback=None):
    """p.iters ADMM iterations from (u, d) (default zeros); returns (x, u, d)."""
    if u is None or d is None:
        u, d = _zeros_state(b, masks)
    u = np.asarray(u, dtype=np.result_type(np.float64, np.asarray(u).dtype))
    d = np.asarray(d, dtype=np.result_type(np.float64, np.asarray(d).dtype))
    x = None
    for k in range(p.iters):
        x, u, d = iterate(b, masks, u, d, p)
        if callback is not None:
            callback(k, x, u, d)
    return x, u, d


def _neighbours(n, NR, zbc):
    if NR == 1:
        return []
    if zbc == "periodic":
        if NR == 2:
            return [1 - n, 1 - n]
        return [(n - 1) % NR, (n + 1) % NR]
    return [k for k in (n - 1, n + 1) if 0 <= k < NR]


def iterate_paper(b, masks, u, d, p):
    """One iteration of Algorithm 1 (gamma on the u-block, Gauss-Seidel in n)."""
    v = xstep(b, u, d, masks, p.rho, 0.0, p.zbc)
    NR = v.shape[0]
    u_new = np.array(u, dtype=np.result_type(u.dtype, v.dtype), copy=True)
    for n in range(NR):
        nb = _neighbours(n, NR, p.zbc)
        wsum = p.rho + p.gamma * len(nb)
        g = p.rho * (v[n] + d[n])
        for k in nb:
            g = g + p.gamma * u_new[k]  # newest value: k < n already updated this sweep
        g = g / wsum
        u_new[n] = denoise(g[None], p, strength_rho=wsum)[0]
    d_new = d + v - u_new
    return v, u_new, d_new


def solve_paper(b, masks, p, u=None, d=None, callback=None):
    if u is None or d is None:
        u, d = _zeros_state(b, masks)
    u = np.asarray(u, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    v = None
    for k in range(p.iters):
        v, u, d = iterate_paper(b, masks, u, d, p)
        if callback is not None:
            callback(k, v, u, d)
    return v, u, d


def objective(v, b, masks, p):
    """Value of the temporal objective at v for the TV or Tikhonov prior."""
    r = np.asarray(b) - forward(v, masks)
    data = 0.5 * np.sum(r * r)
    if p.denoiser == "tikhonov":
        reg = p.lam * np.sum(np.asarray(v) ** 2)
    elif p.denoiser == "tv":
        reg = p.lam * np.sum(tv_value(v))
    else:
        raise ValueError("objective defined for tikhonov and tv priors")
    return data + reg + p.gamma * temporal_energy(v, p.zbc)


__all__ = ["Params", "iterate", "solve", "iterate_paper", "solve_paper", "objective"]
