"""Pins for the oracle's TV prox and Tikhonov closed forms (CPU only).

TV: the discrete divergence is the negative adjoint of the gradient; the
1D two-level step has a textbook ROF solution; the primal-dual gap of the
Chambolle iterate vanishes; constants are fixed points; a huge weight gives
the mean.  Tikhonov: the closed forms of Sec. III-B and Sec. III-C agree with
numeric minimisation.
"""
import numpy as np
import pytest
from scipy.optimize import minimize_scalar

import oracle
from oracle.tv import grad2d, div2d, tv_chambolle, tv_value


def test_div_is_negative_adjoint_of_grad():
    g = np.random.default_rng([11])
    for H, W in [(5, 7), (1, 6), (6, 1), (2, 2), (9, 4)]:
        u = g.normal(size=(H, W))
        px = g.normal(size=(H, W))
        py = g.normal(size=(H, W))
        gx, gy = grad2d(u)
        lhs = np.sum(gx * px + gy * py)
        rhs = -np.sum(u * div2d(px, py))
        assert abs(lhs - rhs) < 1e-12 * max(1, abs(lhs))


def test_div_is_explicit_minus_transpose():
    # build grad as a matrix column by column and compare div with -G^T
    H, W = 3, 4
    n = H * W
    G = np.zeros((2 * n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1
        gx, gy = grad2d(e.reshape(H, W))
        G[:, k] = np.concatenate([gx.ravel(), gy.ravel()])
    D = np.zeros((n, 2 * n))
    for k in range(2 * n):
        e = np.zeros(2 * n)
        e[k] = 1
        D[:, k] = div2d(e[:n].reshape(H, W), e[n:].reshape(H, W)).ravel()
    np.testing.assert_allclose(D, -G.T, atol=0)


@pytest.mark.parametrize("tau", [0.125, 0.25])
@pytest.mark.parametrize("a,c,n1,n2,theta", [(0.0, 1.0, 6, 10, 0.5), (0.2, 0.9, 4, 5, 0.3)])
def test_two_level_step_closed_form(tau, a, c, n1, n2, theta):
    rows = 3
    f = np.concatenate([np.full((rows, n1), a), np.full((rows, n2), c)], axis=1)
    u, px, py = tv_chambolle(f, theta, 20000, tau)
    lo, hi = a + theta / n1, c - theta / n2
    assert lo < hi
    np.testing.assert_allclose(u[:, :n1], lo, atol=1e-10)
    np.testing.assert_allclose(u[:, n1:], hi, atol=1e-10)


def test_duality_gap_vanishes():
    g = np.random.default_rng([12])
    f = g.random((8, 9))
    theta = 0.2
    u, px, py = tv_chambolle(f, theta, 20000, 0.125)
    assert np.all(px * px + py * py <= 1 + 1e-12)
    primal = 0.5 * np.sum((u - f) ** 2) + theta * tv_value(u)
    dual = 0.5 * np.sum(f * f) - 0.5 * np.sum((f - theta * div2d(px, py)) ** 2)
    assert primal - dual >= -1e-12
    assert primal - dual < 1e-8


def test_constant_is_fixed_point_and_large_weight_gives_mean():
    f = np.full((5, 6), 0.37)
    u, _, _ = tv_chambolle(f, 0.4, 17, 0.125)
    np.testing.assert_array_equal(u, f)
    g = np.random.default_rng([13])
    f = g.random((4, 4))
    u, _, _ = tv_chambolle(f, 50.0, 60000, 0.25)
    np.testing.assert_allclose(u, f.mean(), atol=1e-6)


def test_tv_prox_zero_weight_is_identity():
    f = np.random.default_rng([14]).random((3, 4, 5))
    np.testing.assert_array_equal(oracle.tv_prox(f, 0.0, 1.0, 10), f)


def test_tikhonov_closed_forms_match_numeric_minimum():
    g = np.random.default_rng([15])
    for _ in range(10):
        lam, rho, gam = g.uniform(0.01, 2, 3)
        f, a, b = g.normal(size=3)
        # Sec. III-B: argmin lam u^2 + rho/2 (u - f)^2
        num = minimize_scalar(lambda t: lam * t * t + 0.5 * rho * (t - f) ** 2, tol=1e-14).x
        assert abs(oracle.tikhonov(f, lam, rho) - num) < 1e-7
        # Sec. III-C: argmin lam u^2 + rho/2 (u-f)^2 + gam/2 (u-a)^2 + gam/2 (u-b)^2
        num = minimize_scalar(lambda t: lam * t * t + 0.5 * rho * (t - f) ** 2
                              + 0.5 * gam * ((t - a) ** 2 + (t - b) ** 2), tol=1e-14).x
        closed = (rho * f + gam * (a + b)) / (2 * lam + rho + 2 * gam)
        assert abs(closed - num) < 1e-7
        # the paper's temporal step is Tikhonov at rho + 2 gamma on the averaged datum
        avg = (rho * f + gam * (a + b)) / (rho + 2 * gam)
        assert abs(oracle.tikhonov(avg, lam, rho + 2 * gam) - closed) < 1e-14
