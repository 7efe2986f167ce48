"""BM3D u-step on the GPU vs the oracle.

Group membership (the block-matching decision) is taken in FP64 with the same
fixed summation order on both sides, so match lists are compared exactly in
both stages; the FP64 basic estimate to 1e-12; the FP32 output to 1e-6; a
short BM3D + temporal solve to 1e-4.  At the full 1024 x 1024 x 16 size the
stage-1 groups of sampled references are checked exactly."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import announce, rel_l2, to_gpu, to_np
from oracle import bm3d as OB

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cs():
    from paper_2511_03093_amd import cspnp
    assert torch.cuda.is_available()
    cspnp.load()
    return cspnp


def noisy_volume(R, H, W, seed, sigma=0.04):
    g = np.random.default_rng([71, seed])
    vol = np.clip(synth.blob_volume(g, R, H, W, max(3, H * W // 600)), 0, 1)
    return (vol + g.normal(0, sigma, vol.shape)).astype(np.float32)


def stage_outputs(cs, plan, p, f, stage):
    ws = plan.workspace(p, cs.WS_DENOISE)
    cs.cspnp_bm3d_stage(plan._handle, p, f.data_ptr(), stage, plan._ws_ptr(ws), cs._stream())
    torch.cuda.synchronize()
    L = cs.cspnp_bm3d_layout(plan._handle)
    base = plan._ws_ptr(ws) - ws.data_ptr()
    raw = ws.cpu().numpy()[base:]
    NR = plan.R
    nref = NR * L["nry"] * L["nrx"]
    matches = raw[L["matches"]:L["matches"] + nref * 64].view(np.int32).reshape(NR, L["nry"] * L["nrx"], 16)
    counts = raw[L["counts"]:L["counts"] + nref * 4].view(np.int32).reshape(NR, L["nry"] * L["nrx"])
    vol = NR * plan.H * plan.W
    basic = raw[L["basic"]:L["basic"] + vol * 8].view(np.float64).reshape(NR, plan.H, plan.W)
    return matches, counts, basic.copy()


def groups_of(matches, counts, W):
    return [[(int(i) // W, int(i) % W) for i in matches[k, :counts[k]]] for k in range(matches.shape[0])]


@pytest.mark.parametrize("H,W", [(40, 45), (64, 70), (23, 96)])
def test_stage1_matches_basic_and_stage2_matches(cs, H, W):
    announce("bm3d-stages", H, W)
    R = 2
    f = noisy_volume(R, H, W, H)
    sigma = 0.04
    plan = cs.Plan(np.zeros((R, H, W), np.uint8), denoiser="bm3d")
    p = cs.make_params(bm3d_sigma=sigma)
    fg = to_gpu(f)
    m1, c1, _ = stage_outputs(cs, plan, p, fg, 0)
    _, _, basic = stage_outputs(cs, plan, p, fg, 1)
    m2, c2, _ = stage_outputs(cs, plan, p, fg, 2)
    for s in range(R):
        img = f[s].astype(np.float64)
        g1 = OB.match_all(img, OB.TAU_HT)
        assert groups_of(m1[s], c1[s], W) == g1
        bo = OB.stage_ht(img, sigma, g1)
        assert rel_l2(basic[s], bo) < 1e-12
        g2 = OB.match_all(bo, OB.TAU_WIE)
        assert groups_of(m2[s], c2[s], W) == g2


@pytest.mark.parametrize("H,W,sigma", [(48, 56, 0.04), (33, 40, 0.1)])
def test_bm3d_denoise(cs, H, W, sigma):
    announce("bm3d-denoise", H, W, sigma)
    R = 2
    f = noisy_volume(R, H, W, W, sigma)
    plan = cs.Plan(np.zeros((R, H, W), np.uint8), denoiser="bm3d")
    u, d = plan.denoise(cs.make_params(bm3d_sigma=sigma), to_gpu(f))
    uo = OB.bm3d(f, sigma)
    assert rel_l2(to_np(u), uo) < 1e-6
    assert rel_l2(to_np(d), f - uo) < 1e-5


def test_bm3d_temporal_solve(cs):
    announce("bm3d-solve")
    prob = synth.make_problem(40, 48, 4, 1, n_blobs=6, noise=("gauss", 0.02), seed=(72,))
    p = oracle.Params(denoiser="bm3d", lam=0.05, rho=1.0, gamma=0.1, iters=3, bm3d_sigma=9.669 / 255)
    xo, uo, do = oracle.solve(prob.y, prob.masks, p)
    plan = cs.Plan(prob.masks, denoiser="bm3d")
    x, u, d = plan.solve(cs.params_from(p, flags=cs.FLAG_NO_GRAPH), to_gpu(prob.y))
    assert rel_l2(to_np(x), xo) < 1e-4
    assert rel_l2(to_np(u), uo) < 1e-4


def test_full_size_sampled_groups(cs):
    """1024 x 1024 x 16 (the BM3D workload): stage-1 groups of sampled references."""
    announce("bm3d-full-size")
    prob = synth.make(5)
    NR, H, W = prob.gt.shape
    plan = cs.Plan(prob.masks, denoiser="bm3d")
    p = cs.params_from(prob.params)
    # the datum of the first u-step: f = x^1 + d^0 with u = d = 0
    x, f = plan.xupdate(p, to_gpu(prob.y), torch.zeros(prob.gt.shape, device="cuda"),
                        torch.zeros(prob.gt.shape, device="cuda"))
    m1, c1, _ = stage_outputs(cs, plan, p, f, 0)
    fh = to_np(f).astype(np.float64)
    L = cs.cspnp_bm3d_layout(plan._handle)
    rng = np.random.default_rng([73])
    for _ in range(24):
        s = int(rng.integers(NR))
        iy, ix = int(rng.integers(L["nry"])), int(rng.integers(L["nrx"]))
        ry, rx = OB.ref_positions(H)[iy], OB.ref_positions(W)[ix]
        grp = OB.match(fh[s], ry, rx, OB.TAU_HT)
        k = iy * L["nrx"] + ix
        assert groups_of(m1[s, k:k + 1], c1[s, k:k + 1], W)[0] == grp
    # and the full u-step runs on the whole volume
    u, d = plan.denoise(p, f)
    uh = to_np(u)
    assert np.isfinite(uh).all()
