"""Launch shapes change speed only: every TV tile shape and x-update block
shape gives bit-identical results; the autotuner picks valid shapes and
round-trips its JSON cache."""
import json
import os

import numpy as np
import pytest

import synth
from gpu_util import announce, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cs():
    import torch
    from paper_2511_03093_amd import cspnp
    assert torch.cuda.is_available()
    cspnp.load()
    return cspnp


@pytest.mark.parametrize("H,W,inner", [(300, 410, 10), (97, 130, 3), (200, 200, 20)])
def test_shapes_bitwise_identical(cs, H, W, inner):
    announce("shapes", H, W, inner)
    R = 3
    g = np.random.default_rng([21, H, W])
    f = (synth.blob_volume(g, R, H, W, 20) + 0.05 * g.normal(size=(R, H, W))).astype(np.float32)
    y = g.random((1, H, W)).astype(np.float32)
    u0, d0 = synth.random_state((R, H, W), (H, W))
    plan = cs.Plan((g.random((R, H, W)) < 0.5).astype(np.uint8), denoiser="tv")
    p = cs.make_params(lam=0.07, rho=1.0, gamma=0.1, tv_inner=inner)
    nt, nx = cs.cspnp_tuning_candidates()
    ref_u = ref_x = None
    for t in range(nt):
        plan.set_tuning(t, t % nx)
        try:
            u, d = plan.denoise(p, to_gpu(f))
        except cs.CspnpError:
            continue  # halo does not fit this tile
        x, _ = plan.xupdate(p, to_gpu(y), to_gpu(u0), to_gpu(d0), want_f=False)
        u, x = to_np(u), to_np(x)
        if ref_u is None:
            ref_u, ref_x = u, x
        np.testing.assert_array_equal(u, ref_u)
        np.testing.assert_array_equal(x, ref_x)
    assert ref_u is not None


def test_autotune_and_cache(cs, tmp_path):
    announce("autotune")
    prob = synth.make(2, H=256, W=256, n_blobs=20)
    plan = cs.Plan(prob.masks, denoiser="tv")
    p = cs.params_from(prob.params)
    cache = str(tmp_path / "tune.json")
    tv, xu = plan.autotune(p, cache)
    nt, nx = cs.cspnp_tuning_candidates()
    assert 0 <= tv < nt and 0 <= xu < nx
    data = json.load(open(cache))
    assert len(data) == 1
    (key, ent), = data.items()
    assert "256x256/R16" in key and ent["tv_shape"] == tv and ent["xu_block"] == xu
    plan2 = cs.Plan(prob.masks, denoiser="tv")
    plan2.set_tuning((tv + 1) % nt, (xu + 1) % nx)
    assert plan2.autotune(p, cache) == (tv, xu)  # read back from the cache
    with pytest.raises(cs.CspnpError):
        plan2.set_tuning(nt, 0)
