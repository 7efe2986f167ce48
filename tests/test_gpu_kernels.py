"""Kernel-level parity of the HIP path against the FP64 oracle, through the C-ABI.

Operator: adjoint exact, forward <= 1e-6; x-step <= 1e-6 (FP64 internal);
TV prox <= 1e-5 (FP32 arithmetic over 10+ inner iterations); Tikhonov <= 1e-6.
Shapes span several TV tiles (128 x 128 with a halo) and ragged tails.
"""
import numpy as np
import pytest

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


def masks_for(R, H, W, seed, p=0.5):
    return (np.random.default_rng([5, R, H, W, seed]).random((R, H, W)) < p).astype(np.uint8)


@pytest.mark.parametrize("R,H,W", [(8, 64, 64), (16, 33, 77), (1, 5, 3), (24, 40, 100), (32, 17, 64), (3, 1, 1)])
def test_operator(cs, R, H, W):
    announce("operator", R, H, W)
    m = masks_for(R, H, W, 1)
    g = np.random.default_rng([6, R, H, W])
    x = g.normal(size=(R, H, W)).astype(np.float32)
    y = g.normal(size=(1, H, W)).astype(np.float32)
    plan = cs.Plan(m)
    yg = to_np(plan.forward(to_gpu(x)))
    xg = to_np(plan.adjoint(to_gpu(y)))
    assert rel_l2(yg, oracle.forward(x, m)) < 1e-6
    np.testing.assert_array_equal(xg, (m * y).astype(np.float32))
    # adjoint identity on the GPU results
    lhs = float(np.vdot(yg.astype(np.float64), y))
    rhs = float(np.vdot(x.astype(np.float64), xg))
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + 1)


@pytest.mark.parametrize("R", [1, 2, 3, 5, 8, 16, 24, 32])
@pytest.mark.parametrize("zbc", ["periodic", "neumann"])
@pytest.mark.parametrize("rho,gamma", [(1.0, 0.1), (1.0, 0.0), (0.0114, 0.001), (1e-3, 0.5959)])
def test_xupdate(cs, R, zbc, rho, gamma):
    H, W = 37, 70
    announce("xupdate", R, zbc, rho, gamma)
    m = masks_for(R, H, W, 2)
    m[:, 0, 0] = 0
    m[:, 0, 1] = 1
    g = np.random.default_rng([7, R])
    y = g.random((1, H, W)).astype(np.float32) * R / 2
    u = g.random((R, H, W)).astype(np.float32)
    d = (g.normal(size=(R, H, W)) * 0.1).astype(np.float32)
    plan = cs.Plan(m, zbc=zbc)
    p = cs.make_params(lam=0.05, rho=rho, gamma=gamma)
    x, f = plan.xupdate(p, to_gpu(y), to_gpu(u), to_gpu(d))
    xo = oracle.xstep(y, u, d, m, rho, gamma, zbc)
    assert rel_l2(to_np(x), xo) < 1e-6
    assert rel_l2(to_np(f), xo + d) < 1e-6


@pytest.mark.parametrize("H,W", [(64, 64), (300, 260), (129, 257), (7, 200), (1, 1), (2, 300), (512, 512)])
@pytest.mark.parametrize("inner", [0, 1, 10])
def test_tv_prox(cs, H, W, inner):
    R = 2
    announce("tv", H, W, inner)
    g = np.random.default_rng([8, H, W, inner])
    f = synth.blob_volume(g, R, H, W, max(1, H * W // 2000)) + 0.05 * g.normal(size=(R, H, W))
    f = f.astype(np.float32)
    lam, rho = 0.05, 1.0
    plan = cs.Plan(masks_for(R, H, W, 3), denoiser="tv")
    p = cs.make_params(lam=lam, rho=rho, tv_inner=inner)
    u, d = plan.denoise(p, to_gpu(f))
    uo = oracle.tv_prox(f, lam, rho, inner)
    assert rel_l2(to_np(u), uo) < 1e-5
    assert rel_l2(to_np(d), f - uo) < 1e-5 or np.linalg.norm(f - uo) < 1e-6


@pytest.mark.parametrize("inner,theta,tau", [(20, 0.05, 0.125), (37, 0.3, 0.25), (16, 0.1, 0.125), (17, 0.1, 0.125)])
def test_tv_prox_multipass(cs, inner, theta, tau):
    H, W, R = 200, 150, 3
    announce("tv-multipass", inner, theta, tau)
    g = np.random.default_rng([9, inner])
    f = (synth.blob_volume(g, R, H, W, 30) + 0.05 * g.normal(size=(R, H, W))).astype(np.float32)
    plan = cs.Plan(masks_for(R, H, W, 4), denoiser="tv")
    p = cs.make_params(lam=theta, rho=1.0, tv_inner=inner, tv_tau=tau)
    u, d = plan.denoise(p, to_gpu(f))
    uo = oracle.tv_prox(f, theta, 1.0, inner, tau)
    assert rel_l2(to_np(u), uo) < 1e-5


def test_tv_zero_weight_is_identity(cs):
    H, W, R = 50, 60, 2
    f = np.random.default_rng([10]).random((R, H, W)).astype(np.float32)
    plan = cs.Plan(masks_for(R, H, W, 5), denoiser="tv")
    u, d = plan.denoise(cs.make_params(lam=0.0, rho=1.0, tv_inner=10), to_gpu(f))
    np.testing.assert_array_equal(to_np(u), f)
    np.testing.assert_array_equal(to_np(d), np.zeros_like(f))


def test_tikhonov(cs):
    H, W, R = 45, 70, 4
    f = np.random.default_rng([11]).normal(size=(R, H, W)).astype(np.float32)
    plan = cs.Plan(masks_for(R, H, W, 6), denoiser="tikhonov")
    u, d = plan.denoise(cs.make_params(lam=0.3, rho=0.7), to_gpu(f))
    uo = oracle.tikhonov(f.astype(np.float64), 0.3, 0.7)
    assert rel_l2(to_np(u), uo) < 1e-6
    assert rel_l2(to_np(d), f - uo) < 1e-6


def test_param_validation_on_device(cs):
    H, W, R = 8, 8, 2
    plan = cs.Plan(masks_for(R, H, W, 7), denoiser="tv")
    f = to_gpu(np.zeros((R, H, W), np.float32))
    for bad in [dict(rho=0.0), dict(rho=-1.0), dict(lam=-0.1), dict(gamma=-1.0), dict(tv_inner=-1),
                dict(tv_tau=0.3), dict(tv_tau=0.0), dict(rho=float("nan"))]:
        with pytest.raises(cs.CspnpError) as ei:
            plan.denoise(cs.make_params(**bad), f)
        assert ei.value.status == cs.EINVAL
    with pytest.raises(cs.CspnpError):
        plan.xupdate(cs.make_params(iters=-1), f[:1], f, f)
