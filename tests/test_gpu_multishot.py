"""N > 1 shots per volume (the paper reconstructs 40 frames from N = 40/R coded
shots): block-elimination x-step, operator, full solves and Algorithm 1's own
schedule against the oracle; PSNR across compression ratios."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import announce, rel_l2, to_gpu, to_np
from oracle import metrics as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cs():
    from paper_2511_03093_amd import cspnp
    assert torch.cuda.is_available()
    cspnp.load()
    return cspnp


@pytest.mark.parametrize("N,R", [(2, 1), (2, 4), (3, 2), (5, 8), (4, 10), (2, 20), (8, 5)])
@pytest.mark.parametrize("zbc", ["periodic", "neumann"])
@pytest.mark.parametrize("rho,gamma", [(1.0, 0.1), (0.01, 0.6), (1.0, 0.0)])
def test_multishot_xstep(cs, N, R, zbc, rho, gamma):
    announce("multishot-xstep", N, R, zbc, rho, gamma)
    H, W = 19, 37
    g = np.random.default_rng([111, N, R])
    masks = (g.random((R, H, W)) < 0.5).astype(np.uint8)
    masks[:, 0, 0] = 0
    y = (g.random((N, H, W)) * R / 2).astype(np.float32)
    u = g.random((N * R, H, W)).astype(np.float32)
    d = (g.normal(size=(N * R, H, W)) * 0.1).astype(np.float32)
    plan = cs.Plan(masks, N=N, zbc=zbc)
    x, f = plan.xupdate(cs.make_params(rho=rho, gamma=gamma), to_gpu(y), to_gpu(u), to_gpu(d))
    xo = oracle.xstep(y, u, d, masks, rho, gamma, zbc)
    assert rel_l2(to_np(x), xo) < 1e-6
    assert rel_l2(to_np(f), xo + d) < 1e-6


def test_multishot_operator(cs):
    N, R, H, W = 5, 8, 33, 50
    g = np.random.default_rng([112])
    masks = (g.random((R, H, W)) < 0.5).astype(np.uint8)
    x = g.normal(size=(N * R, H, W)).astype(np.float32)
    y = g.normal(size=(N, H, W)).astype(np.float32)
    plan = cs.Plan(masks, N=N)
    assert rel_l2(to_np(plan.forward(to_gpu(x))), oracle.forward(x, masks)) < 1e-6
    np.testing.assert_array_equal(to_np(plan.adjoint(to_gpu(y))), oracle.adjoint(y, masks).astype(np.float32))


@pytest.mark.parametrize("schedule", ["default", "paper"])
def test_multishot_solve_40_frames(cs, schedule):
    """200 x 200 pixels, 40 frames from N = 5 shots of R = 8 (the paper's volume size)."""
    announce("multishot-solve", schedule)
    prob = synth.make_problem(200, 200, 8, 5, n_blobs=60, noise=("gauss", 0.01), seed=(113,))
    p = oracle.Params(denoiser="tv", lam=0.05, rho=1.0, gamma=0.1, iters=8, tv_inner=10)
    if schedule == "paper":
        xo, uo, do = oracle.solve_paper(prob.y, prob.masks, p)
        flags = cs.FLAG_PAPER_SCHEDULE
    else:
        xo, uo, do = oracle.solve(prob.y, prob.masks, p)
        flags = 0
    plan = cs.Plan(prob.masks, N=5, denoiser="tv")
    x, u, d = plan.solve(cs.params_from(p, flags=flags), to_gpu(prob.y))
    assert rel_l2(to_np(x), xo) < 1e-4
    assert rel_l2(to_np(u), uo) < 1e-4


def test_psnr_falls_with_compression_ratio(cs):
    """Fig. 4's trend on synthetic data: 40 frames, fewer measurements as R grows."""
    announce("cr-sweep")
    rng = np.random.default_rng([114])
    gt = np.clip(synth.blob_volume(rng, 40, 128, 128, 80), 0, 1).astype(np.float32)
    scores = {}
    for R in (2, 8, 20):
        N = 40 // R
        masks = synth.bernoulli_masks(np.random.default_rng([115, R]), R, 128, 128)
        y = synth.simulate_frames(gt.astype(np.float64), masks, N, R).astype(np.float32)
        plan = cs.Plan(masks, N=N, denoiser="tv")
        x, _, _ = plan.solve(cs.make_params(lam=0.02, rho=1.0, gamma=0.1, iters=60), to_gpu(y))
        scores[R] = M.psnr(to_np(x), gt)
    assert scores[2] > scores[8] > scores[20], scores


@pytest.mark.parametrize("N,R,zbc", [(32, 32, "periodic"), (1024, 1, "neumann"), (64, 16, "periodic")])
def test_maximum_depth(cs, N, R, zbc):
    """The deepest volume a plan accepts (N*R = 1024 slices): x-step and a short TV solve."""
    announce("max-depth", N, R, zbc)
    H, W = 4, 5
    g = np.random.default_rng([116, N, R])
    masks = (g.random((R, H, W)) < 0.5).astype(np.uint8)
    y = (g.random((N, H, W)) * R / 2).astype(np.float32)
    u = g.random((N * R, H, W)).astype(np.float32)
    d = (g.normal(size=(N * R, H, W)) * 0.1).astype(np.float32)
    plan = cs.Plan(masks, N=N, zbc=zbc, denoiser="tv")
    x, _ = plan.xupdate(cs.make_params(rho=0.5, gamma=0.3), to_gpu(y), to_gpu(u), to_gpu(d))
    xo = oracle.xstep(y, u, d, masks, 0.5, 0.3, zbc)
    assert rel_l2(to_np(x), xo) < 1e-6
    p = oracle.Params(denoiser="tv", lam=0.05, rho=1.0, gamma=0.1, iters=3, tv_inner=5, zbc=zbc)
    xo, uo, _ = oracle.solve(y, masks, p)
    xg, ug, _ = plan.solve(cs.params_from(p), to_gpu(y))
    assert rel_l2(to_np(xg), xo) < 1e-4
    assert rel_l2(to_np(ug), uo) < 1e-4
