"""Gradient-based choice of the ADMM parameters (rho, lambda, gamma).

The paper picks these three numbers per prior by Bayesian optimisation of the
reconstruction quality on data with a known ground truth (Sec. IV-B).  Here
the same choice is made by gradient descent: Adam on the logarithms of the
parameters, minimising the mean squared error of x^K against the reference
volume, with the gradients of the library's differentiable solve
(``cspnp_solve_ckpt`` / ``cspnp_solve_bwd`` through :mod:`.autograd`).  Every
solve and every gradient runs in the library; this module only holds the
three scalars and the optimiser state.
"""
from __future__ import annotations

import math

import torch

from .autograd import pnp_admm


def tune(plan, y, x_ref, rho, lam, gamma, iters, steps=20, lr=0.15, tv_inner=10, ckpt_every=5,
         tune_gamma=True):
    """Adam on (log rho, log lambda, log gamma) for ``steps`` evaluations.

    y: device frames of the plan; x_ref: device reference volume.  gamma = 0
    (or tune_gamma=False) keeps gamma fixed.  Returns (best, history): best is
    the evaluated point of lowest loss, history one dict per evaluation with
    the loss and the parameters it was evaluated at.
    """
    dev = y.device
    logs = {"rho": torch.tensor(math.log(rho), dtype=torch.float64, device=dev, requires_grad=True),
            "lam": torch.tensor(math.log(lam), dtype=torch.float64, device=dev, requires_grad=True)}
    if tune_gamma and gamma > 0:
        logs["gamma"] = torch.tensor(math.log(gamma), dtype=torch.float64, device=dev, requires_grad=True)
    opt = torch.optim.Adam(list(logs.values()), lr=lr)
    n = x_ref.numel()
    history = []
    best = None
    for s in range(steps):
        opt.zero_grad()
        r = torch.exp(logs["rho"])
        l = torch.exp(logs["lam"])
        g = torch.exp(logs["gamma"]) if "gamma" in logs else gamma
        x = pnp_admm(y, r, l, g, plan, iters=iters, tv_inner=tv_inner, ckpt_every=ckpt_every)
        loss = torch.sum((x.double() - x_ref.double()) ** 2) / n
        loss.backward()
        gv = float(g.detach()) if isinstance(g, torch.Tensor) else float(g)
        rec = {"step": s, "loss": float(loss.detach()), "rho": float(r.detach()), "lam": float(l.detach()),
               "gamma": gv}
        history.append(rec)
        if best is None or rec["loss"] < best["loss"]:
            best = rec
        opt.step()
    return best, history
