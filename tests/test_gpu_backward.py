"""The hand-written backward through the unrolled iterations, via the C-ABI.

GPU gradient vs the oracle's FP64 reverse mode: rel <= 1e-4 (scalars and
y_bar); GPU gradient vs FP32 central differences of the GPU forward (step
1e-3) at the full 512 x 512 x 16, 30-iteration workload: rel <= 1e-2.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import announce, rel_l2, to_gpu, to_np
from oracle.grad import mse_grad, solve_vjp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cs():
    from paper_2511_03093_amd import cspnp
    assert torch.cuda.is_available()
    cspnp.load()
    return cspnp


def gpu_vjp(cs, plan, p, y, xbar, c):
    """(x^K, ybar, [rho, lam, gamma]) from the C-ABI."""
    shape = plan.vol_shape
    u = torch.zeros(shape, device="cuda")
    d = torch.zeros(shape, device="cuda")
    x = torch.empty(shape, device="cuda")
    ckpt = torch.empty(cs.cspnp_ckpt_size(plan._handle, p, c) // 4, device="cuda")
    ws = plan.workspace(p)
    cs.cspnp_solve_ckpt(plan._handle, p, y.data_ptr(), u.data_ptr(), d.data_ptr(), x.data_ptr(), c, ckpt.data_ptr(),
                        plan._ws_ptr(ws), cs._stream())
    ybar = torch.empty_like(y)
    pbar = torch.empty(3, dtype=torch.float64, device="cuda")
    nb = cs.cspnp_bwd_workspace_size(plan._handle, p, c)
    wsb = torch.empty(nb + 256, dtype=torch.uint8, device="cuda")
    cs.cspnp_solve_bwd(plan._handle, p, y.data_ptr(), c, ckpt.data_ptr(), xbar.data_ptr(), ybar.data_ptr(),
                       pbar.data_ptr(), plan._ws_ptr(wsb), cs._stream())
    return to_np(x), to_np(ybar), to_np(pbar)


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-30)


@pytest.mark.parametrize("denoiser,zbc,gamma", [("tv", "periodic", 0.1), ("tv", "neumann", 0.2),
                                                ("tv", "periodic", 0.0), ("tikhonov", "periodic", 0.1)])
@pytest.mark.parametrize("c", [3, 7])
def test_vjp_matches_oracle(cs, denoiser, zbc, gamma, c):
    announce("vjp", denoiser, zbc, gamma, c)
    prob = synth.make_problem(48, 40, 8, 1, n_blobs=8, seed=(41, c))
    p = oracle.Params(denoiser=denoiser, lam=0.05, rho=1.0, gamma=gamma, iters=7, tv_inner=10, zbc=zbc)
    xbar = np.random.default_rng([42]).normal(size=prob.gt.shape).astype(np.float32)
    ref = solve_vjp(prob.y, prob.masks, p, xbar.astype(np.float64))
    plan = cs.Plan(prob.masks, zbc=zbc, denoiser=denoiser)
    x, ybar, pbar = gpu_vjp(cs, plan, cs.params_from(p), to_gpu(prob.y), to_gpu(xbar), c)
    assert rel_l2(x, ref["x"]) < 1e-4
    assert rel_l2(ybar, ref["y"]) < 1e-4
    assert rel(pbar[0], ref["rho"]) < 1e-4
    assert rel(pbar[1], ref["lam"]) < 1e-4
    if gamma > 0 or zbc == "periodic":
        assert rel(pbar[2], ref["gamma"]) < 1e-4


@pytest.mark.parametrize("N,R,zbc,gamma", [(2, 8, "periodic", 0.1), (3, 4, "neumann", 0.2), (5, 8, "periodic", 0.1),
                                          (2, 1, "periodic", 0.3)])
def test_multishot_vjp_matches_oracle(cs, N, R, zbc, gamma):
    announce("vjp-multishot", N, R, zbc, gamma)
    prob = synth.make_problem(40, 36, R, N, n_blobs=8, seed=(43, N, R))
    p = oracle.Params(denoiser="tv", lam=0.05, rho=1.0, gamma=gamma, iters=6, tv_inner=10, zbc=zbc)
    xbar = np.random.default_rng([44]).normal(size=prob.gt.shape).astype(np.float32)
    ref = solve_vjp(prob.y, prob.masks, p, xbar.astype(np.float64))
    plan = cs.Plan(prob.masks, N=N, zbc=zbc, denoiser="tv")
    x, ybar, pbar = gpu_vjp(cs, plan, cs.params_from(p), to_gpu(prob.y), to_gpu(xbar), 4)
    assert rel_l2(x, ref["x"]) < 1e-4
    assert rel_l2(ybar, ref["y"]) < 1e-4
    assert rel(pbar[0], ref["rho"]) < 1e-4
    assert rel(pbar[1], ref["lam"]) < 1e-4
    assert rel(pbar[2], ref["gamma"]) < 1e-4


def test_checkpoint_interval_and_determinism(cs):
    announce("ckpt-interval")
    prob = synth.make_problem(64, 72, 8, 1, n_blobs=8, seed=(43,))
    p = cs.make_params(lam=0.05, rho=1.0, gamma=0.1, iters=6, tv_inner=10)
    plan = cs.Plan(prob.masks, denoiser="tv")
    xbar = to_gpu(np.random.default_rng([44]).normal(size=prob.gt.shape))
    y = to_gpu(prob.y)
    outs = [gpu_vjp(cs, plan, p, y, xbar, c) for c in (1, 4, 6, 6)]
    for o in outs[1:]:
        np.testing.assert_array_equal(o[1], outs[0][1])
        np.testing.assert_array_equal(o[2], outs[0][2])


def test_autograd_mse_matches_oracle_reduced(cs):
    """TV + temporal, B = 16, 30 unrolled iterations, checkpoint every 5, at 128 x 128."""
    announce("autograd-reduced")
    from paper_2511_03093_amd.autograd import pnp_admm
    prob = synth.make(4, H=128, W=128, n_blobs=20)
    p = oracle.Params.from_dict(prob.params)
    ref = mse_grad(prob.y, prob.masks, p, prob.gt.astype(np.float64))
    plan = cs.Plan(prob.masks, denoiser="tv")
    y = to_gpu(prob.y).requires_grad_(True)
    rho = torch.tensor(p.rho, dtype=torch.float64, requires_grad=True)
    lam = torch.tensor(p.lam, dtype=torch.float64, requires_grad=True)
    gam = torch.tensor(p.gamma, dtype=torch.float64, requires_grad=True)
    x = pnp_admm(y, rho, lam, gam, plan, iters=p.iters, tv_inner=p.tv_inner, ckpt_every=5)
    loss = torch.mean((x.double() - to_gpu(prob.gt).double()) ** 2)
    loss.backward()
    assert rel(float(loss), ref["loss"]) < 1e-4
    assert rel(float(rho.grad), ref["rho"]) < 1e-4
    assert rel(float(lam.grad), ref["lam"]) < 1e-4
    assert rel(float(gam.grad), ref["gamma"]) < 1e-4
    assert rel_l2(to_np(y.grad), ref["y"]) < 1e-4


def test_full_size_gradients_vs_central_differences(cs):
    """512 x 512 x 16, 30 iterations, checkpoint every 5: FP32 central differences, step 1e-3."""
    announce("full-size-fd")
    from paper_2511_03093_amd.autograd import pnp_admm
    prob = synth.make(4)
    pd = prob.params
    plan = cs.Plan(prob.masks, denoiser="tv")
    gt = to_gpu(prob.gt).double()
    y0 = to_gpu(prob.y)

    def loss_at(y, rho, lam, gam):
        x = pnp_admm(y, rho, lam, gam, plan, iters=pd["iters"], tv_inner=pd["tv_inner"], ckpt_every=5)
        return torch.mean((x.double() - gt) ** 2)

    y = y0.clone().requires_grad_(True)
    sc = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in (pd["rho"], pd["lam"], pd["gamma"])]
    loss = loss_at(y, *sc)
    loss.backward()
    h = 1e-3
    with torch.no_grad():
        base = [pd["rho"], pd["lam"], pd["gamma"]]
        for k in range(3):
            up = list(base)
            dn = list(base)
            up[k] += h
            dn[k] -= h
            fd = (float(loss_at(y0, *up)) - float(loss_at(y0, *dn))) / (2 * h)
            assert rel(float(sc[k].grad), fd) < 1e-2, (k, float(sc[k].grad), fd)
        v = torch.from_numpy(np.random.default_rng([45]).choice([-1.0, 1.0], size=prob.y.shape).astype(np.float32)).cuda()
        fd = (float(loss_at(y0 + h * v, *base)) - float(loss_at(y0 - h * v, *base))) / (2 * h)
        an = float(torch.sum(y.grad.double() * v.double()))
        assert rel(an, fd) < 1e-2, (an, fd)


def test_bwd_graph_replay_equals_direct_launch(cs):
    """The captured backward (first call captures, the second replays) equals direct launches bit for bit."""
    announce("bwd-graph")
    prob = synth.make_problem(64, 72, 8, 1, n_blobs=6, seed=(47, 1))
    p = oracle.Params(denoiser="tv", lam=0.05, rho=1.0, gamma=0.1, iters=6, tv_inner=10, zbc="periodic")
    plan = cs.Plan(prob.masks, zbc="periodic", denoiser="tv")
    y = to_gpu(prob.y)
    xbar = to_gpu(np.random.default_rng([48]).normal(size=prob.gt.shape).astype(np.float32))
    runs = [gpu_vjp(cs, plan, cs.params_from(p), y, xbar, 4) for _ in range(2)]
    direct = gpu_vjp(cs, plan, cs.params_from(p, flags=cs.FLAG_NO_GRAPH), y, xbar, 4)
    for r in runs[1:] + [direct]:
        for a, b in zip(r, runs[0]):
            np.testing.assert_array_equal(a, b)
