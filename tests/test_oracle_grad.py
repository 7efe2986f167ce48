"""Pins for the oracle's reverse-mode gradient (CPU only).

The hand-written adjoint is compared with complex-step derivatives of the
forward oracle (Im l(t + i h)/h, h = 1e-30: exact to rounding, no
cancellation) and with central finite differences.
"""
import numpy as np
import pytest

import oracle
from oracle.grad import mse_grad, solve_vjp, tv_vjp
from oracle.tv import tv_chambolle
from synth import make_problem


def loss_of(prob, p, y=None):
    y = prob.y if y is None else y
    x, _, _ = oracle.solve(y, prob.masks, p)
    return np.mean((x - prob.gt) ** 2)


H_CS = 1e-30


def cs_deriv(fn, t0):
    return np.imag(fn(t0 + 1j * H_CS)) / H_CS


@pytest.mark.parametrize("denoiser", ["tv", "tikhonov"])
@pytest.mark.parametrize("zbc,gamma", [("periodic", 0.1), ("neumann", 0.3), ("periodic", 0.0)])
def test_gradient_matches_complex_step(denoiser, zbc, gamma):
    prob = make_problem(9, 11, 4, 1, n_blobs=3, seed=(31, int(gamma * 10)))
    p = oracle.Params(denoiser=denoiser, lam=0.05, rho=0.8, gamma=gamma, iters=4, tv_inner=5, zbc=zbc)
    g = mse_grad(prob.y, prob.masks, p, prob.gt)
    d_rho = cs_deriv(lambda t: loss_of(prob, p.with_(rho=t)), p.rho)
    d_lam = cs_deriv(lambda t: loss_of(prob, p.with_(lam=t)), p.lam)
    assert abs(g["rho"] - d_rho) <= 1e-9 * max(abs(d_rho), 1e-12) + 1e-15
    assert abs(g["lam"] - d_lam) <= 1e-9 * max(abs(d_lam), 1e-12) + 1e-15
    if gamma > 0:
        d_gam = cs_deriv(lambda t: loss_of(prob, p.with_(gamma=t)), p.gamma)
        assert abs(g["gamma"] - d_gam) <= 1e-9 * max(abs(d_gam), 1e-12) + 1e-15
    v = np.random.default_rng([32]).choice([-1.0, 1.0], size=prob.y.shape)
    d_y = cs_deriv(lambda t: loss_of(prob, p, prob.y.astype(np.float64) + t * v), 0.0)
    assert abs(np.sum(g["y"] * v) - d_y) <= 1e-9 * abs(d_y) + 1e-15


def test_gradient_matches_central_differences():
    prob = make_problem(8, 8, 3, 1, n_blobs=2, seed=(33,))
    p = oracle.Params(denoiser="tv", lam=0.06, rho=1.0, gamma=0.1, iters=3, tv_inner=4)
    g = mse_grad(prob.y, prob.masks, p, prob.gt)
    h = 1e-6
    for name in ("rho", "lam", "gamma"):
        t = getattr(p, name)
        fd = (loss_of(prob, p.with_(**{name: t + h})) - loss_of(prob, p.with_(**{name: t - h}))) / (2 * h)
        assert abs(g[name] - fd) <= 1e-5 * abs(fd) + 1e-12


def test_tv_vjp_alone():
    rng = np.random.default_rng([34])
    f = rng.random((2, 7, 6))
    ubar = rng.normal(size=f.shape)
    theta, n, tau = 0.2, 6, 0.125
    fbar, thetabar = tv_vjp(f, theta, n, tau, ubar)
    d_theta = cs_deriv(lambda t: np.sum(ubar * tv_chambolle(f, t, n, tau)[0]), theta)
    assert abs(thetabar - d_theta) < 1e-10 * abs(d_theta) + 1e-14
    v = rng.normal(size=f.shape)
    d_f = cs_deriv(lambda t: np.sum(ubar * tv_chambolle(f + t * v, theta, n, tau)[0]), 0.0)
    assert abs(np.sum(fbar * v) - d_f) < 1e-10 * abs(d_f) + 1e-14


def test_vjp_is_linear_in_xbar():
    prob = make_problem(6, 7, 3, 1, n_blobs=2, seed=(35,))
    p = oracle.Params(denoiser="tv", lam=0.05, rho=1.0, gamma=0.1, iters=3, tv_inner=3)
    rng = np.random.default_rng([36])
    a, b = rng.normal(size=prob.gt.shape), rng.normal(size=prob.gt.shape)
    ga = solve_vjp(prob.y, prob.masks, p, a)
    gb = solve_vjp(prob.y, prob.masks, p, b)
    gab = solve_vjp(prob.y, prob.masks, p, 2 * a - b)
    for k in ("rho", "lam", "gamma"):
        assert abs(gab[k] - (2 * ga[k] - gb[k])) < 1e-10 * (abs(ga[k]) + abs(gb[k]) + 1e-12)
    np.testing.assert_allclose(gab["y"], 2 * ga["y"] - gb["y"], rtol=1e-9, atol=1e-13)


@pytest.mark.parametrize("zbc", ["periodic", "neumann"])
def test_gradient_multishot_matches_complex_step(zbc):
    # N = 2 shots: the temporal chain couples the two shots' slices
    prob = make_problem(7, 9, 3, 2, n_blobs=3, seed=(37, len(zbc)))
    p = oracle.Params(denoiser="tv", lam=0.05, rho=0.9, gamma=0.2, iters=3, tv_inner=4, zbc=zbc)
    g = mse_grad(prob.y, prob.masks, p, prob.gt)
    for name in ("rho", "lam", "gamma"):
        t = getattr(p, name)
        d = cs_deriv(lambda s: loss_of(prob, p.with_(**{name: s})), t)
        assert abs(g[name] - d) <= 1e-9 * max(abs(d), 1e-12) + 1e-15
    v = np.random.default_rng([38]).choice([-1.0, 1.0], size=prob.y.shape)
    d_y = cs_deriv(lambda t: loss_of(prob, p, prob.y.astype(np.float64) + t * v), 0.0)
    assert abs(np.sum(g["y"] * v) - d_y) <= 1e-9 * abs(d_y) + 1e-15
