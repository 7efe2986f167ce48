"""Gradient-based parameter choice (Adam on log rho, log lambda, log gamma
through the differentiable solve): it lowers the reconstruction error from a
poor start, and the point it reports reproduces its loss in a fresh solve.
The gradients themselves are checked against the oracle in test_gpu_backward."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import announce, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cs():
    from paper_2511_03093_amd import cspnp
    assert torch.cuda.is_available()
    cspnp.load()
    return cspnp


@pytest.mark.parametrize("N,R", [(1, 8), (2, 4)])
def test_tuning_lowers_the_error(cs, N, R):
    from paper_2511_03093_amd.tune import tune
    announce("tune", N, R)
    prob = synth.make_problem(64, 56, R, N, n_blobs=10, seed=(51, N, R))
    plan = cs.Plan(prob.masks, N=N, denoiser="tv")
    y, gt = to_gpu(prob.y), to_gpu(prob.gt)
    best, hist = tune(plan, y, gt, rho=1.0, lam=0.2, gamma=0.5, iters=20, steps=12, lr=0.2)
    assert len(hist) == 12
    assert best["loss"] < 0.7 * hist[0]["loss"], (best, hist[0])
    # the reported point reproduces its loss
    x, _, _ = plan.solve(cs.make_params(lam=best["lam"], rho=best["rho"], gamma=best["gamma"], iters=20), y)
    mse = float(np.mean((to_np(x).astype(np.float64) - prob.gt) ** 2))
    assert abs(mse - best["loss"]) <= 1e-5 * best["loss"]


def test_fixed_gamma_stays_fixed(cs):
    from paper_2511_03093_amd.tune import tune
    announce("tune-fixed-gamma")
    prob = synth.make_problem(48, 48, 8, 1, n_blobs=8, seed=(52,))
    plan = cs.Plan(prob.masks, denoiser="tv")
    best, hist = tune(plan, to_gpu(prob.y), to_gpu(prob.gt), rho=1.0, lam=0.1, gamma=0.0, iters=10, steps=4)
    assert all(h["gamma"] == 0.0 for h in hist)
    assert best["loss"] <= hist[0]["loss"]
