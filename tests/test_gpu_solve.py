"""Solve-level parity of the HIP path against the FP64 oracle, through the C-ABI.

Per iteration (from the oracle's own state, rounded to FP32): rel L2 of x, u,
d <= 1e-5.  Free-running full solve: rel L2 of x <= 1e-4.  Plus structural
properties: graph replay == direct launches bit for bit, run-to-run
determinism, and resuming from a saved (u, d) state.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import announce, rel_l2, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cs():
    import torch
    from paper_2511_03093_amd import cspnp
    assert torch.cuda.is_available()
    cspnp.load()
    return cspnp


def oparams(prob, **over):
    p = oracle.Params.from_dict(prob.params)
    return p.with_(**over) if over else p


@pytest.mark.parametrize("denoiser", ["tv", "tikhonov"])
@pytest.mark.parametrize("zbc,gamma", [("periodic", 0.1), ("neumann", 0.1), ("periodic", 0.0)])
def test_one_iteration_from_oracle_state(cs, denoiser, zbc, gamma):
    announce("iteration", denoiser, zbc, gamma)
    prob = synth.make(2, H=160, W=144, B=16, n_blobs=40)
    p = oparams(prob, denoiser=denoiser, zbc=zbc, gamma=gamma, iters=3)
    _, uo, do = oracle.solve(prob.y, prob.masks, p)
    u32, d32 = uo.astype(np.float32), do.astype(np.float32)
    x1, u1, d1 = oracle.iterate(prob.y, prob.masks, u32.astype(np.float64), d32.astype(np.float64), p)
    plan = cs.Plan(prob.masks, zbc=zbc, denoiser=denoiser)
    x, u, d = plan.solve(cs.params_from(p, iters=1), to_gpu(prob.y), to_gpu(u32), to_gpu(d32))
    assert rel_l2(to_np(x), x1) < 1e-5
    assert rel_l2(to_np(u), u1) < 1e-5
    assert rel_l2(to_np(d), d1) < 1e-5


def test_full_solve_workload1(cs):
    """256 x 256, B = 8, TV, gamma = 0, 50 iterations (full size)."""
    announce("full-solve", "256x256x8 TV 50 it")
    prob = synth.make(1)
    p = oparams(prob)
    xo, uo, do = oracle.solve(prob.y, prob.masks, p)
    plan = cs.Plan(prob.masks, zbc=p.zbc, denoiser=p.denoiser)
    x, u, d = plan.solve(cs.params_from(p), to_gpu(prob.y))
    assert rel_l2(to_np(x), xo) < 1e-4
    assert rel_l2(to_np(u), uo) < 1e-4


def test_full_solve_workload2_reduced(cs):
    """TV + temporal (0.1, periodic), B = 16, 100 iterations, at 128 x 128."""
    announce("full-solve", "128x128x16 TV+temporal 100 it")
    prob = synth.make(2, H=128, W=128, n_blobs=20)
    p = oparams(prob)
    xo, uo, do = oracle.solve(prob.y, prob.masks, p)
    plan = cs.Plan(prob.masks, zbc=p.zbc, denoiser=p.denoiser)
    x, u, d = plan.solve(cs.params_from(p), to_gpu(prob.y))
    assert rel_l2(to_np(x), xo) < 1e-4
    assert rel_l2(to_np(u), uo) < 1e-4


def test_workload2_full_size_first_iterations(cs):
    """512 x 512, B = 16 (the benchmark's launch configuration): 3 iterations."""
    announce("full-size", "512x512x16 3 it")
    prob = synth.make(2)
    p = oparams(prob, iters=3)
    xo, uo, do = oracle.solve(prob.y, prob.masks, p)
    plan = cs.Plan(prob.masks, zbc=p.zbc, denoiser=p.denoiser)
    x, u, d = plan.solve(cs.params_from(p), to_gpu(prob.y))
    assert rel_l2(to_np(x), xo) < 1e-5
    assert rel_l2(to_np(u), uo) < 1e-5


def test_graph_replay_equals_direct_launch_and_is_deterministic(cs):
    announce("graph-replay")
    prob = synth.make(2, H=200, W=180, n_blobs=30)
    p = oparams(prob, iters=7)
    plan = cs.Plan(prob.masks, zbc=p.zbc, denoiser=p.denoiser)
    y = to_gpu(prob.y)
    shape = prob.gt.shape
    outs = []
    for flags in (cs.FLAG_NO_GRAPH, 0, 0):
        u = torch.zeros(shape, device="cuda")
        d = torch.zeros(shape, device="cuda")
        x = torch.empty(shape, device="cuda")
        ws = plan.workspace(cs.params_from(p))
        plan.solve(cs.params_from(p, flags=flags), y, u, d, x, ws)
        outs.append((to_np(x), to_np(u), to_np(d)))
    for a, b in zip(outs[0], outs[1]):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(outs[1], outs[2]):
        np.testing.assert_array_equal(a, b)
    # replay on identical buffers (cached graph) several times with eager work between
    u = torch.zeros(shape, device="cuda")
    d = torch.zeros(shape, device="cuda")
    x = torch.empty(shape, device="cuda")
    ws = plan.workspace(cs.params_from(p))
    for rep in range(3):
        u.zero_()
        d.zero_()
        plan.solve(cs.params_from(p), y, u, d, x, ws)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(to_np(x), outs[0][0])
        np.testing.assert_array_equal(to_np(u), outs[0][1])


def test_resume_equals_continuous(cs):
    announce("resume")
    prob = synth.make(2, H=96, W=130, n_blobs=10)
    p = oparams(prob)
    plan = cs.Plan(prob.masks, zbc=p.zbc, denoiser=p.denoiser)
    y = to_gpu(prob.y)
    x, u, d = plan.solve(cs.params_from(p, iters=9), y)
    u2 = torch.zeros_like(u)
    d2 = torch.zeros_like(d)
    plan.solve(cs.params_from(p, iters=4), y, u2, d2)
    x2, u2, d2 = plan.solve(cs.params_from(p, iters=5), y, u2, d2)
    np.testing.assert_array_equal(to_np(x), to_np(x2))
    np.testing.assert_array_equal(to_np(u), to_np(u2))


@pytest.mark.parametrize("H,W,R", [(1, 1, 1), (3, 5, 2), (1, 300, 4), (300, 1, 3), (70, 33, 32)])
def test_degenerate_shapes(cs, H, W, R):
    announce("degenerate", H, W, R)
    prob = synth.make_problem(H, W, R, 1, n_blobs=2, seed=(77, H, W, R))
    p = oracle.Params(denoiser="tv", lam=0.05, rho=1.0, gamma=0.1, iters=6, tv_inner=10)
    xo, uo, do = oracle.solve(prob.y, prob.masks, p)
    plan = cs.Plan(prob.masks, denoiser="tv")
    x, u, d = plan.solve(cs.params_from(p), to_gpu(prob.y))
    assert rel_l2(to_np(x), xo) < 1e-4


@pytest.mark.parametrize("fill", [0, 1])
def test_all_closed_or_all_open_masks(cs, fill):
    announce("mask-fill", fill)
    prob = synth.make_problem(40, 50, 6, 1, n_blobs=5, seed=(78, fill))
    masks = np.full_like(prob.masks, fill)
    y = synth.simulate_frames(prob.gt.astype(np.float64), masks, 1, 6).astype(np.float32)
    p = oracle.Params(denoiser="tv", lam=0.05, rho=1.0, gamma=0.1, iters=5)
    xo, _, _ = oracle.solve(y, masks, p)
    plan = cs.Plan(masks, denoiser="tv")
    x, _, _ = plan.solve(cs.params_from(p), to_gpu(y))
    if fill == 0:
        np.testing.assert_array_equal(to_np(x), np.zeros_like(xo))
    else:
        assert rel_l2(to_np(x), xo) < 1e-4


def test_zero_iterations_leave_state(cs):
    prob = synth.make_problem(20, 20, 4, 1, n_blobs=2, seed=(79,))
    plan = cs.Plan(prob.masks, denoiser="tv")
    u0, d0 = synth.random_state(prob.gt.shape, (1,))
    x, u, d = plan.solve(cs.make_params(iters=0), to_gpu(prob.y), to_gpu(u0), to_gpu(d0))
    np.testing.assert_array_equal(to_np(u), u0)
    np.testing.assert_array_equal(to_np(d), d0)
