"""Batched solves: every batched result equals its unbatched solve bit for bit
(same per-pixel and per-tile arithmetic), on a mixed mini-batch and on the
full 64-snapshot workload; one snapshot is also checked against the oracle."""
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


def plain(cs, masks, p, y):
    plan = cs.Plan(masks, denoiser="tv")
    x, u, d = plan.solve(p, y)
    torch.cuda.synchronize()
    plan.close()
    return x, u, d


def test_mixed_minibatch_equals_unbatched(cs):
    announce("minibatch")
    shapes = [(64, 64, 8), (100, 130, 16), (77, 200, 3), (256, 256, 8), (130, 97, 24), (33, 45, 1), (300, 260, 16)]
    probs = [synth.make_problem(H, W, R, 1, n_blobs=6, seed=(51, i)) for i, (H, W, R) in enumerate(shapes)]
    rng = np.random.default_rng([52])
    params = [cs.make_params(lam=float(rng.uniform(0.02, 0.1)), rho=float(rng.uniform(0.5, 2)),
                             gamma=float(rng.uniform(0, 0.3)), iters=9, tv_inner=int(rng.integers(3, 12)))
              for _ in shapes]
    batch = cs.Batch([p.masks for p in probs])
    y = [to_gpu(p.y) for p in probs]
    for rep in range(2):  # second call replays the cached graph
        u, d, x = batch.allocate()
        batch.solve(params, y, u, d, x)
        torch.cuda.synchronize()
        for i, pr in enumerate(probs):
            xr, ur, dr = plain(cs, pr.masks, params[i], y[i])
            assert torch.equal(x[i], xr) and torch.equal(u[i], ur) and torch.equal(d[i], dr), (rep, i)
    # one snapshot against the oracle
    i = 1
    op = oracle.Params(denoiser="tv", lam=params[i].lambda_, rho=params[i].rho, gamma=params[i].gamma, iters=9,
                       tv_inner=params[i].tv_inner)
    xo, _, _ = oracle.solve(probs[i].y, probs[i].masks, op)
    assert rel_l2(to_np(x[i]), xo) < 1e-4


def test_every_tv_shape_same_result(cs):
    announce("batch-shapes")
    probs = [synth.make_problem(H, W, R, 1, n_blobs=4, seed=(53, i))
             for i, (H, W, R) in enumerate([(90, 150, 8), (200, 120, 16)])]
    p = [cs.make_params(lam=0.05, rho=1.0, gamma=0.1, iters=4, tv_inner=10)] * 2
    batch = cs.Batch([q.masks for q in probs])
    y = [to_gpu(q.y) for q in probs]
    ref = None
    for s in range(cs.cspnp_tuning_candidates()[0]):
        cs.cspnp_batch_set_tv_shape(batch._handle, s)
        u, d, x = batch.allocate()
        batch.solve(p, y, u, d, x)
        out = [to_np(t) for t in x]
        if ref is None:
            ref = out
        for a, b in zip(out, ref):
            np.testing.assert_array_equal(a, b)


def test_full_64_snapshot_batch_equals_unbatched(cs):
    """The batched workload: 64 snapshots, sizes {256^2, 512^2, 768x512, 1024^2}, B in {8,16,24}, 100 iterations."""
    announce("batch-64")
    probs = [synth.make(3, snapshot=s) for s in range(64)]
    pd = probs[0].params
    params = [cs.params_from(pd)] * 64
    batch = cs.Batch([p.masks for p in probs])
    y = [to_gpu(p.y) for p in probs]
    u, d, x = batch.allocate()
    batch.solve(params, y, u, d, x)
    torch.cuda.synchronize()
    for i, pr in enumerate(probs):
        xr, ur, dr = plain(cs, pr.masks, params[i], y[i])
        assert torch.equal(x[i], xr) and torch.equal(u[i], ur), i
