"""torch.autograd.Function around the library's differentiable solve.

``PnPADMM.apply(y, rho, lam, gamma, plan, settings)`` returns x^K (the last
x-step of ``settings['iters']`` iterations from u = d = 0); its backward calls
``cspnp_solve_bwd`` (checkpointed recomputation, hand-written adjoint kernels)
and returns gradients for y and for the three scalar tensors.  Argument
marshalling only; no arithmetic of the method runs in Python.
"""
from __future__ import annotations

import torch

from . import cspnp


def _ws(nbytes):
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    return t, (t.data_ptr() + 255) & ~255


def _scalar(t):
    return float(t.detach()) if isinstance(t, torch.Tensor) else float(t)


class PnPADMM(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, rho, lam, gamma, plan, settings):
        c = int(settings.get("ckpt_every", 5))
        p = cspnp.make_params(lam=_scalar(lam), rho=_scalar(rho), gamma=_scalar(gamma), iters=settings["iters"],
                              tv_inner=settings.get("tv_inner", 10), tv_tau=settings.get("tv_tau", 0.125))
        y = y.contiguous()
        shape = plan.vol_shape
        u = torch.zeros(shape, dtype=torch.float32, device="cuda")
        d = torch.zeros(shape, dtype=torch.float32, device="cuda")
        x = torch.empty(shape, dtype=torch.float32, device="cuda")
        ckpt = torch.empty(cspnp.cspnp_ckpt_size(plan._handle, p, c) // 4, dtype=torch.float32, device="cuda")
        ws_t, ws = _ws(cspnp.cspnp_workspace_size(plan._handle, p, cspnp.WS_SOLVE))
        cspnp.cspnp_solve_ckpt(plan._handle, p, y.data_ptr(), u.data_ptr(), d.data_ptr(), x.data_ptr(), c,
                               ckpt.data_ptr(), ws, cspnp._stream())
        ctx.plan, ctx.p, ctx.c = plan, p, c
        ctx.save_for_backward(y, ckpt)
        ctx.scalar_meta = [(t.dtype, t.device) if isinstance(t, torch.Tensor) else None for t in (rho, lam, gamma)]
        return x

    @staticmethod
    def backward(ctx, xbar):
        y, ckpt = ctx.saved_tensors
        plan, p, c = ctx.plan, ctx.p, ctx.c
        xbar = xbar.contiguous().to(torch.float32)
        ybar = torch.empty_like(y)
        pbar = torch.empty(3, dtype=torch.float64, device="cuda")
        ws_t, ws = _ws(cspnp.cspnp_bwd_workspace_size(plan._handle, p, c))
        cspnp.cspnp_solve_bwd(plan._handle, p, y.data_ptr(), c, ckpt.data_ptr(), xbar.data_ptr(), ybar.data_ptr(),
                              pbar.data_ptr(), ws, cspnp._stream())
        outs = []
        for k, meta in enumerate(ctx.scalar_meta):
            outs.append(None if meta is None else pbar[k].to(dtype=meta[0], device=meta[1]))
        return (ybar, outs[0], outs[1], outs[2], None, None)


def pnp_admm(y, rho, lam, gamma, plan, **settings):
    return PnPADMM.apply(y, rho, lam, gamma, plan, settings)
