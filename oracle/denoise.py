"""Plug-and-play denoisers of the u-step (oracle).

The u-step denoises f = v + d at strength lambda/rho (Sec. III-B, eq. (u-sub)):

* Tikhonov, psi(u) = ||u||^2: closed form u = rho f / (2 lambda + rho);
* TV: Chambolle's dual projection with theta = lambda/rho, cold-started at
  p = 0 on every call, tv_inner iterations of step tv_tau;
* BM3D: see :mod:`oracle.bm3d` (its strength is a noise level, not lambda).
"""
from .tv import tv_chambolle


def tikhonov(f, lam, rho):
    return rho * f / (2.0 * lam + rho)


def tv_prox(f, lam, rho, n_iter, tau=0.125):
    u, _, _ = tv_chambolle(f, lam / rho, n_iter, tau)
    return u


def denoise(f, params, strength_rho=None):
    """Apply the configured denoiser to f (all slices).  ``strength_rho`` replaces rho in
    the strength lambda/rho (the paper's temporal schedule uses rho + 2 gamma)."""
    rho = params.rho if strength_rho is None else strength_rho
    if params.denoiser == "tikhonov":
        return tikhonov(f, params.lam, rho)
    if params.denoiser == "tv":
        return tv_prox(f, params.lam, rho, params.tv_inner, params.tv_tau)
    if params.denoiser == "bm3d":
        from .bm3d import bm3d
        return bm3d(f, params.bm3d_sigma)
    raise ValueError(f"unknown denoiser {params.denoiser!r}")
