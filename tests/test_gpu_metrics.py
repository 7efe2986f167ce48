"""On-GPU quality metrics and the relative-tolerance stopping rule vs the oracle."""
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


@pytest.mark.parametrize("D,H,W", [(13, 40, 50), (11, 11, 11), (16, 64, 33)])
def test_metrics_match_oracle(cs, D, H, W):
    announce("metrics", D, H, W)
    rng = np.random.default_rng([101, D, H, W])
    ref = np.clip(synth.blob_volume(rng, D, H, W, 6), 0, 1).astype(np.float32)
    est = np.clip(ref + rng.normal(0, 0.05, ref.shape), 0, 1).astype(np.float32)
    e, r = to_gpu(est), to_gpu(ref)
    assert abs(cs.psnr(e, r) - M.psnr(est, ref)) < 1e-9
    assert abs(cs.psnr(e, r, 2.0) - M.psnr(est, ref, 2.0)) < 1e-9
    assert abs(cs.ssim(e, r, 2) - M.ssim2d(est, ref)) < 1e-10
    assert abs(cs.ssim(e, r, 3) - M.ssim3d(est, ref)) < 1e-10
    assert abs(cs.ssim(r, r, 3) - 1.0) < 1e-12
    assert abs(cs.rel_change(e, r) - M.rel_change(est, ref)) < 1e-12


def test_solve_tol_stops_like_the_oracle_and_equals_plain_solve(cs):
    announce("solve-tol")
    prob = synth.make(2, H=96, W=80, n_blobs=12)
    p = oracle.Params.from_dict(prob.params).with_(iters=200)
    tol = 2e-3
    rels = []
    xprev = [None]

    def cb(k, x, u, d):
        if xprev[0] is not None:
            rels.append(M.rel_change(x, xprev[0]))
        xprev[0] = x.copy()

    oracle.solve(prob.y, prob.masks, p.with_(iters=60), callback=cb)
    k_oracle = next(i + 2 for i, r in enumerate(rels) if r < tol)
    plan = cs.Plan(prob.masks, denoiser="tv")
    x, u, d, it, rel = plan.solve_tol(cs.params_from(p), to_gpu(prob.y), tol, check_every=1)
    assert abs(it - k_oracle) <= 1 and rel < tol
    xr, ur, dr = plan.solve(cs.params_from(p, iters=it), to_gpu(prob.y))
    assert torch.equal(x, xr) and torch.equal(u, ur) and torch.equal(d, dr)
    # a coarser test interval stops at the first multiple of check_every past the threshold
    x5, _, _, it5, rel5 = plan.solve_tol(cs.params_from(p), to_gpu(prob.y), tol, check_every=5)
    assert it5 % 5 == 0 and it5 >= it and rel5 < tol


def test_reconstruction_beats_backprojection(cs):
    announce("quality")
    prob = synth.make(2, H=128, W=128, n_blobs=40)
    plan = cs.Plan(prob.masks, denoiser="tv")
    gt = to_gpu(prob.gt)
    x1, _, _ = plan.solve(cs.params_from(prob.params, iters=1), to_gpu(prob.y))
    x, _, _ = plan.solve(cs.params_from(prob.params), to_gpu(prob.y))
    assert cs.psnr(x, gt) > cs.psnr(x1, gt) + 3.0
    assert cs.ssim(x, gt) > cs.ssim(x1, gt)
