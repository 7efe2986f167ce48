"""Algorithm 1's own schedule (temporal term on the u-block, Gauss-Seidel
sweep over slices) on the GPU vs the oracle's solve_paper."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import announce, rel_l2, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cs():
    from paper_2511_03093_amd import cspnp
    assert torch.cuda.is_available()
    cspnp.load()
    return cspnp


@pytest.mark.parametrize("denoiser", ["tv", "tikhonov"])
@pytest.mark.parametrize("zbc,R", [("periodic", 8), ("neumann", 8), ("periodic", 2), ("periodic", 1), ("neumann", 3)])
def test_paper_schedule_matches_oracle(cs, denoiser, zbc, R):
    announce("paper-schedule", denoiser, zbc, R)
    prob = synth.make_problem(70, 90, R, 1, n_blobs=10, seed=(81, R))
    p = oracle.Params(denoiser=denoiser, lam=0.05, rho=1.0, gamma=0.2, iters=6, tv_inner=10, zbc=zbc)
    vo, uo, do = oracle.solve_paper(prob.y, prob.masks, p)
    plan = cs.Plan(prob.masks, zbc=zbc, denoiser=denoiser)
    x, u, d = plan.solve(cs.params_from(p, flags=cs.FLAG_PAPER_SCHEDULE), to_gpu(prob.y))
    assert rel_l2(to_np(x), vo) < 1e-4
    assert rel_l2(to_np(u), uo) < 1e-4
    assert rel_l2(to_np(d), do) < 1e-4


def test_paper_schedule_one_iteration_from_oracle_state(cs):
    announce("paper-schedule-iteration")
    prob = synth.make(2, H=128, W=96, n_blobs=20)
    p = oracle.Params.from_dict(prob.params).with_(iters=3)
    _, uo, do = oracle.solve_paper(prob.y, prob.masks, p)
    u32, d32 = uo.astype(np.float32), do.astype(np.float32)
    v1, u1, d1 = oracle.iterate_paper(prob.y, prob.masks, u32.astype(np.float64), d32.astype(np.float64), p)
    plan = cs.Plan(prob.masks, denoiser="tv")
    x, u, d = plan.solve(cs.params_from(p, iters=1, flags=cs.FLAG_PAPER_SCHEDULE), to_gpu(prob.y), to_gpu(u32),
                         to_gpu(d32))
    assert rel_l2(to_np(x), v1) < 1e-5
    assert rel_l2(to_np(u), u1) < 1e-5
    assert rel_l2(to_np(d), d1) < 1e-5


def test_paper_schedule_equals_default_at_gamma0(cs):
    """The note closing Algorithm 1: with gamma = 0 the two schedules coincide."""
    announce("paper-schedule-gamma0")
    prob = synth.make_problem(64, 80, 8, 1, n_blobs=8, seed=(82,))
    plan = cs.Plan(prob.masks, denoiser="tv")
    p = cs.make_params(lam=0.05, rho=1.0, gamma=0.0, iters=5)
    xa, ua, da = plan.solve(p, to_gpu(prob.y))
    pp = cs.make_params(lam=0.05, rho=1.0, gamma=0.0, iters=5, flags=cs.FLAG_PAPER_SCHEDULE)
    xb, ub, db = plan.solve(pp, to_gpu(prob.y))
    assert rel_l2(to_np(xb), to_np(xa)) < 1e-6
    assert rel_l2(to_np(ub), to_np(ua)) < 1e-6
