"""Differentiable link travel times: a torch.autograd.Function over the HIP
simulator.

``IDMTravelTime.apply(theta, scen, steps, checkpoint_every)`` runs a fresh
simulation of ``scen`` for ``steps`` steps with per-class IDM parameters
``theta`` [num_classes, 4] = (v0_scale, T, a, b) (Sec. 6.3.2, car-following
equation) and returns the mean crossing-interpolated travel time of every link
(Sec. 6.4), in seconds.  Its backward calls the library's adjoint (sim_grad):
the gradient of the travel times with the window's discrete events held fixed,
computed by checkpoint-and-recompute.
"""
from __future__ import annotations

import torch

from . import Sim


class IDMTravelTime(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, scen, steps, checkpoint_every=60, device=0):
        sc = dict(scen)
        sc["params"] = dict(scen["params"])
        sc["params"]["idm"] = theta.detach().to("cpu", torch.float32).numpy().reshape(-1, 4)
        sim = Sim(sc, device=device)
        sim.tape_begin(checkpoint_every)
        sim.step(int(steps))
        tbar, cnt = sim.mean_travel_times()
        ctx.sim = sim
        ctx.theta_device = theta.device
        ctx.mark_non_differentiable(cnt)
        return tbar, cnt

    @staticmethod
    def backward(ctx, g_tbar, g_cnt):
        dtheta = ctx.sim.grad(g_tbar)
        return dtheta.to(ctx.theta_device), None, None, None, None


def travel_time_loss(tbar, cnt, target):
    """Mean squared error of the mean link travel times over links with at
    least one completed traversal."""
    m = cnt > 0
    d = tbar[m] - target[m]
    return (d * d).mean()
