"""Reverse-mode derivative of the unrolled ADMM (oracle).

The paper defines no gradient; this module differentiates the oracle's own
iteration (:func:`oracle.admm.iterate`: x-step with the temporal term, u-step,
d-step) with respect to the measured frames y, the ADMM penalty rho, the
prior weight lambda and the temporal weight gamma, for a loss of the final
x.  It is written step by step from the forward definitions:

x-step   x = A^{-1} (M^T y + rho (u - d)),  A = M^T M + gamma L + rho I (symmetric):
         with lam_v = A^{-1} xbar:  ybar += M lam_v,  ubar = rho lam_v,  dbar -= rho lam_v,
         rhobar += <lam_v, u - d - x>,  gammabar -= <lam_v, L x>.
f = x + d;  u' = D_theta(f), theta = lambda/rho;  d' = f - u'.
TV step  (Chambolle, p^0 = 0):  w = div p - f/theta,  g = grad w,  s = 1 + tau |g|,
         p' = (p + tau g)/s,  u = f - theta div p^K.  Reverse of one inner step:
         gbar = (tau/s) (pbar' - (pbar'.p') g/|g|)   (g/|g| := 0 where g = 0),
         wbar = -div gbar,  pbar = pbar'/s - grad wbar,  fbar -= wbar/theta,
         thetabar += <wbar, f/theta^2>;  final step: fbar += ubar,
         pbar^K = theta grad ubar,  thetabar -= <ubar, div p^K>.
Tikhonov u = rho f/(2 lambda + rho).
"""
import numpy as np

from .laplacian import zlaplacian
from .operator import forward
from .tv import div2d, grad2d
from .xstep import xstep


def _zeros(b, masks):
    R = np.asarray(masks).shape[0]
    N, H, W = np.asarray(b).shape
    return np.zeros((N * R, H, W)), np.zeros((N * R, H, W))


def tv_forward_tape(f, theta, n_iter, tau):
    """Chambolle iterates p^0..p^K (p^0 = 0) and the output u."""
    px = np.zeros_like(f)
    py = np.zeros_like(f)
    tape = [(px, py)]
    for _ in range(n_iter):
        w = div2d(px, py) - f / theta
        gx, gy = grad2d(w)
        s = 1.0 + tau * np.sqrt(gx * gx + gy * gy)
        px = (px + tau * gx) / s
        py = (py + tau * gy) / s
        tape.append((px, py))
    u = f - theta * div2d(px, py)
    return u, tape


def tv_vjp(f, theta, n_iter, tau, ubar):
    """(fbar, thetabar) of u = TV_theta(f) for the cotangent ubar."""
    if theta == 0:
        return ubar.copy(), 0.0
    _, tape = tv_forward_tape(f, theta, n_iter, tau)
    pKx, pKy = tape[-1]
    fbar = ubar.copy()
    thetabar = -np.sum(ubar * div2d(pKx, pKy))
    gux, guy = grad2d(ubar)
    pbx, pby = theta * gux, theta * guy
    for t in range(n_iter - 1, -1, -1):
        px, py = tape[t]
        qx, qy = tape[t + 1]
        w = div2d(px, py) - f / theta
        gx, gy = grad2d(w)
        mag = np.sqrt(gx * gx + gy * gy)
        s = 1.0 + tau * mag
        a = pbx * qx + pby * qy
        with np.errstate(divide="ignore", invalid="ignore"):
            nx = np.where(mag > 0, gx / np.where(mag > 0, mag, 1.0), 0.0)
            ny = np.where(mag > 0, gy / np.where(mag > 0, mag, 1.0), 0.0)
        gbx = (tau / s) * (pbx - a * nx)
        gby = (tau / s) * (pby - a * ny)
        wbar = -div2d(gbx, gby)
        gwx, gwy = grad2d(wbar)
        pbx = pbx / s - gwx
        pby = pby / s - gwy
        fbar = fbar - wbar / theta
        thetabar = thetabar + np.sum(wbar * f) / theta ** 2
    return fbar, thetabar


def _lap_apply(x, zbc):
    L = zlaplacian(x.shape[0], zbc)
    return np.einsum("ij,jhw->ihw", L, x)


def solve_vjp(b, masks, p, xbar, u0=None, d0=None):
    """Gradient of <xbar, x^K> (x^K: the last x-step of p.iters iterations from (u0, d0)).

    Returns dict(y=..., rho=..., lam=..., gamma=..., x=x^K)."""
    b = np.asarray(b, dtype=np.float64)
    if u0 is None or d0 is None:
        u0, d0 = _zeros(b, masks)
    K = p.iters
    states = []  # (u^k, d^k, x^{k+1}, f^{k+1})
    u, d = np.asarray(u0, np.float64), np.asarray(d0, np.float64)
    x = None
    for k in range(K):
        x = xstep(b, u, d, masks, p.rho, p.gamma, p.zbc)
        f = x + d
        if p.denoiser == "tv":
            un, _ = tv_forward_tape(f, p.lam / p.rho, p.tv_inner, p.tv_tau)
        elif p.denoiser == "tikhonov":
            un = p.rho * f / (2 * p.lam + p.rho)
        else:
            raise ValueError("gradient implemented for tv and tikhonov")
        states.append((u, d, x, f))
        u, d = un, f - un
    ybar = np.zeros_like(b)
    rhobar = lambar = gambar = 0.0
    thetabar = 0.0
    ubar = np.zeros_like(u)
    dbar = np.zeros_like(d)
    theta = p.lam / p.rho
    for k in range(K - 1, -1, -1):
        uk, dk, xk, fk = states[k]
        # d' = f - u',  u' = D(f)
        fbar = dbar.copy()
        uprime_bar = ubar - dbar
        if k < K - 1:
            if p.denoiser == "tv":
                fb, tb = tv_vjp(fk, theta, p.tv_inner, p.tv_tau, uprime_bar)
                fbar += fb
                thetabar += tb
            else:
                c = p.rho / (2 * p.lam + p.rho)
                fbar += c * uprime_bar
                lambar += np.sum(uprime_bar * fk) * (-2 * p.rho / (2 * p.lam + p.rho) ** 2)
                rhobar += np.sum(uprime_bar * fk) * (2 * p.lam / (2 * p.lam + p.rho) ** 2)
        # f = x + d^k
        xb = fbar + (xbar if k == K - 1 else 0.0)
        dbar_k = fbar.copy()
        # x = A^{-1}(M^T y + rho (u - d)):  lam_v = A^{-1} xb  (A symmetric; rho' = rho, rhs 0)
        zero = np.zeros_like(b)
        lam_v = xstep(zero, xb, np.zeros_like(xb), masks, p.rho, p.gamma, p.zbc) / p.rho
        ybar += forward(lam_v, masks)
        ubar = p.rho * lam_v
        dbar = dbar_k - p.rho * lam_v
        rhobar += np.sum(lam_v * (uk - dk - xk))
        gambar -= np.sum(lam_v * _lap_apply(xk, p.zbc))
    if p.denoiser == "tv":
        lambar += thetabar / p.rho
        rhobar -= thetabar * p.lam / p.rho ** 2
    return dict(y=ybar, rho=rhobar, lam=lambar, gamma=gambar, x=x)


def mse_grad(b, masks, p, x_gt):
    """Loss mean((x^K - x_gt)^2) and its gradients (dict keys y, rho, lam, gamma, loss)."""
    from .admm import solve
    x, _, _ = solve(b, masks, p)
    xbar = 2.0 * (x - x_gt) / x.size
    g = solve_vjp(b, masks, p, xbar)
    g["loss"] = float(np.mean((x - x_gt) ** 2))
    return g
