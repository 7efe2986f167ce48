"""Pins for the oracle's ADMM loops (CPU only).

* Tikhonov + temporal ADMM converges to the minimiser of the objective,
  computed by a global dense solve of its normal equations;
* the fixed-point residual ||u^{k+1}-u^k||^2 + ||d^{k+1}-d^k||^2 never grows
  when the sub-problems are solved exactly (He & Yuan, non-ergodic ADMM);
* at gamma = 0 both schedules coincide (the note at the end of Algorithm 1);
* the paper's Gauss-Seidel schedule reaches the same minimiser;
* K1 + K2 iterations resumed from the saved state equal K1 + K2 at once.
"""
import numpy as np
import pytest

import oracle
from oracle import Params
from synth import make_problem

from test_oracle_operator_xstep import explicit_phi, laplacian_chain


def tiny(H=4, W=5, R=4, N=1, seed=0, noise=("gauss", 0.01)):
    return make_problem(H, W, R, N, n_blobs=3, noise=noise, seed=(900, seed))


def direct_tikhonov(prob, p):
    N = prob.y.shape[0]
    NR, H, W = prob.gt.shape
    Phi = explicit_phi(prob.masks, N)
    P = H * W
    A = Phi.T @ Phi + 2 * p.lam * np.eye(NR * P) + p.gamma * np.kron(laplacian_chain(NR, p.zbc), np.eye(P))
    return np.linalg.solve(A, Phi.T @ prob.y.astype(np.float64).reshape(-1)).reshape(NR, H, W)


@pytest.mark.parametrize("zbc", ["periodic", "neumann"])
@pytest.mark.parametrize("gamma", [0.0, 0.3])
@pytest.mark.parametrize("N", [1, 2])
def test_tikhonov_admm_converges_to_direct_solve(zbc, gamma, N):
    prob = tiny(N=N, seed=N)
    p = Params(denoiser="tikhonov", lam=0.05, rho=0.5, gamma=gamma, iters=600, zbc=zbc)
    x, u, d = oracle.solve(prob.y, prob.masks, p)
    ref = direct_tikhonov(prob, p)
    np.testing.assert_allclose(x, ref, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(u, ref, rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("zbc", ["periodic", "neumann"])
def test_paper_schedule_converges_to_same_minimiser(zbc):
    prob = tiny(seed=5)
    p = Params(denoiser="tikhonov", lam=0.05, rho=0.5, gamma=0.3, iters=800, zbc=zbc)
    v, u, d = oracle.solve_paper(prob.y, prob.masks, p)
    ref = direct_tikhonov(prob, p)
    np.testing.assert_allclose(u, ref, rtol=1e-8, atol=1e-9)


@pytest.mark.parametrize("denoiser", ["tikhonov", "tv"])
def test_schedules_identical_at_gamma0(denoiser):
    prob = tiny(H=6, W=7, R=3, seed=6)
    p = Params(denoiser=denoiser, lam=0.05, rho=1.0, gamma=0.0, iters=1, tv_inner=10)
    x1, u1, d1 = oracle.solve(prob.y, prob.masks, p.with_(iters=7))
    x2, u2, d2 = oracle.solve_paper(prob.y, prob.masks, p.with_(iters=7))
    np.testing.assert_allclose(x1, x2, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(u1, u2, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(d1, d2, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("denoiser,inner", [("tikhonov", 0), ("tv", 3000)])
def test_fixed_point_residual_is_monotone(denoiser, inner):
    prob = tiny(H=6, W=6, R=4, seed=7)
    p = Params(denoiser=denoiser, lam=0.05, rho=1.0, gamma=0.1, iters=1, tv_inner=inner)
    u, d = np.zeros(prob.gt.shape), np.zeros(prob.gt.shape)
    res = []
    for k in range(40 if denoiser == "tv" else 120):
        _, u2, d2 = oracle.iterate(prob.y, prob.masks, u, d, p)
        res.append(np.sum((u2 - u) ** 2) + np.sum((d2 - d) ** 2))
        u, d = u2, d2
    res = np.array(res)
    floor = 1e-24 if denoiser == "tikhonov" else 1e-14
    for a, b in zip(res[:-1], res[1:]):
        assert b <= a * (1 + 1e-9) + floor


def test_resume_equals_continuous_run():
    prob = tiny(H=5, W=6, R=4, seed=8)
    p = Params(denoiser="tv", lam=0.05, rho=1.0, gamma=0.1, tv_inner=10)
    x, u, d = oracle.solve(prob.y, prob.masks, p.with_(iters=9))
    _, ua, da = oracle.solve(prob.y, prob.masks, p.with_(iters=4))
    xb, ub, db = oracle.solve(prob.y, prob.masks, p.with_(iters=5), u=ua, d=da)
    np.testing.assert_array_equal(x, xb)
    np.testing.assert_array_equal(u, ub)
    np.testing.assert_array_equal(d, db)


def test_tv_admm_decreases_objective_and_improves_on_backprojection():
    prob = tiny(H=16, W=16, R=4, seed=9, noise=("none",))
    p = Params(denoiser="tv", lam=0.02, rho=1.0, gamma=0.1, iters=200, tv_inner=50)
    x, u, d = oracle.solve(prob.y, prob.masks, p)
    x1, _, _ = oracle.solve(prob.y, prob.masks, p.with_(iters=1))
    assert oracle.objective(u, prob.y, prob.masks, p) < oracle.objective(x1, prob.y, prob.masks, p)
    err = np.linalg.norm(u - prob.gt) / np.linalg.norm(prob.gt)
    err1 = np.linalg.norm(x1 - prob.gt) / np.linalg.norm(prob.gt)
    assert err < err1
