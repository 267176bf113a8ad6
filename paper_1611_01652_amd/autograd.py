"""torch.autograd bridge: forward = `rollout`, backward = `rollout_grad`.

The checkpoint buffer written by the forward launch is kept in the autograd
context, so the backward recomputes each segment from it (the paper unrolls
the whole trajectory instead, section 2.1.1; memory here is O(T / K_ck)).
"""
from __future__ import annotations

import torch


class Rollout(torch.autograd.Function):
    """loss_env = Rollout.apply(sim, x0, u) with x0 [18,B], u [T_max,J]."""

    @staticmethod
    def forward(ctx, sim, x0, u):
        x0 = x0.detach().contiguous()
        u = u.detach().contiguous()
        out = sim.rollout(x0, u, want_ckpt=True, want_final=False)
        ctx.sim = sim
        ctx.save_for_backward(x0, u, out["ckpt"])
        ctx.flags = out["flags"]
        return out["loss"].clone()

    @staticmethod
    def backward(ctx, dloss):
        x0, u, ckpt = ctx.saved_tensors
        g = ctx.sim.rollout_grad(x0, u, ckpt, dloss.detach().contiguous().float())
        gu = g["g_u"] if u.numel() == g["g_u"].numel() else torch.zeros_like(u)
        return None, g["g_x0"].reshape(x0.shape), gu.reshape(u.shape)


def rollout_loss(sim, x0, u):
    return Rollout.apply(sim, x0, u)
