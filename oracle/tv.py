"""Isotropic total variation and Chambolle's dual projection algorithm (oracle).

The u-step of the ADMM is the proximal map of (lambda/rho) psi (Sec. III-B,
eq. (u-sub)); for the TV prior the paper cites Chambolle's algorithm.  With
theta = lambda/rho, the prox solves

    min_u  1/2 ||u - f||^2 + theta TV(u),   TV(u) = sum_ij |(grad u)_ij|,

by the dual fixed point of Chambolle (J. Math. Imaging Vis. 20, 2004), with
the discrete gradient and divergence defined there:

    (grad u)^x_ij = u_{i,j+1} - u_ij  (0 on the last column),
    (grad u)^y_ij = u_{i+1,j} - u_ij  (0 on the last row),
    div = -grad^T  (backward differences with Chambolle's boundary cases),
    p <- (p + tau grad(div p - f/theta)) / (1 + tau |grad(div p - f/theta)|),
    u  = f - theta div p.

Arrays are [..., H, W]; leading axes (slices) are independent.
"""
import numpy as np


def grad2d(u):
    """Forward differences; returns (gx, gy) with Neumann (zero) last column/row."""
    u = np.asarray(u)
    gx = np.zeros_like(u)
    gy = np.zeros_like(u)
    gx[..., :, :-1] = u[..., :, 1:] - u[..., :, :-1]
    gy[..., :-1, :] = u[..., 1:, :] - u[..., :-1, :]
    return gx, gy


def _div_axis(p, axis):
    # Chambolle's case definition along one axis of length n:
    #   first index: p_0, interior: p_i - p_{i-1}, last index: -p_{n-2}
    p = np.moveaxis(np.asarray(p), axis, -1)
    n = p.shape[-1]
    out = np.zeros_like(p)
    if n == 1:
        return np.moveaxis(out, -1, axis)
    out[..., 0] = p[..., 0]
    out[..., 1:n - 1] = p[..., 1:n - 1] - p[..., 0:n - 2]
    out[..., n - 1] = -p[..., n - 2]
    return np.moveaxis(out, -1, axis)


def div2d(px, py):
    """Discrete divergence, the negative adjoint of :func:`grad2d`."""
    return _div_axis(px, -1) + _div_axis(py, -2)


def _mag(gx, gy):
    # sqrt written out (not abs) so complex-step perturbations propagate
    return np.sqrt(gx * gx + gy * gy)


def tv_value(u):
    gx, gy = grad2d(u)
    return np.sum(_mag(gx, gy), axis=(-2, -1))


def tv_chambolle(f, theta, n_iter, tau=0.125, p0=None):
    """Chambolle's dual iteration started from p0 (default 0); returns (u, px, py)."""
    f = np.asarray(f)
    dt = np.result_type(np.float64, f.dtype, type(theta))
    f = f.astype(dt)
    if p0 is None:
        px = np.zeros_like(f)
        py = np.zeros_like(f)
    else:
        px, py = (np.array(a, dtype=dt) for a in p0)
    if theta == 0:
        return f.copy(), px, py
    for _ in range(n_iter):
        w = div2d(px, py) - f / theta
        gx, gy = grad2d(w)
        s = 1.0 + tau * _mag(gx, gy)
        px = (px + tau * gx) / s
        py = (py + tau * gy) / s
    u = f - theta * div2d(px, py)
    return u, px, py
