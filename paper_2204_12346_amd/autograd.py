"""torch.autograd face of the cost: forward = sird_loss with a checkpoint
workspace (the discrete adjoint's forward pass, which saves the state every
ckpt_interval steps), backward = sird_loss_backward from that workspace (the
reverse sweep only), both in the library's HIP kernels.  Loss plus gradient
therefore integrates the window once."""
from __future__ import annotations

import torch

from .core import Batch, sird_loss, sird_loss_backward, sird_loss_backward_workspace

class SirdLoss(torch.autograd.Function):
    """loss = SirdLoss.apply(theta, batch, obs, kind, ckpt_interval)

    theta: theta-shaped float64 device tensor of the batch (requires_grad).
    Returns the particle-indexed losses.  backward() gives
    grad_theta = upstream_grad[p] * dL_p/dtheta in the theta layout.
    ckpt_interval None (or 0) takes the library's default: per problem the
    whole days whose states fit the reverse sweep's LDS slice.  The workspace
    holding the forward pass lives until the graph is freed.
    """

    @staticmethod
    def forward(ctx, theta, batch: Batch, obs, kind="ssre", ckpt_interval=None):
        if theta.dtype != torch.float64:
            raise TypeError(f"SirdLoss: theta must be float64, got {theta.dtype}")
        ci = 0 if ckpt_interval is None else int(ckpt_interval)
        theta_c = theta.detach().contiguous()
        ws = torch.empty(max(sird_loss_backward_workspace(batch, ci), 8), dtype=torch.uint8,
                         device=batch.device)
        loss = sird_loss(batch, theta_c, obs, kind, workspace=ws, ckpt_interval=ci)
        ctx.save_for_backward(theta_c, obs, ws)
        ctx.batch = batch
        ctx.kind = kind
        ctx.ckpt_interval = ci
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        theta, obs, ws = ctx.saved_tensors
        g = grad_loss.detach().to(torch.float64).contiguous()
        grad, _ = sird_loss_backward(ctx.batch, theta, obs, ctx.kind, grad_loss=g,
                                     ckpt_interval=ctx.ckpt_interval, workspace=ws,
                                     from_forward=True)
        return grad, None, None, None, None


def sird_loss_autograd(theta, batch: Batch, obs, kind="ssre", ckpt_interval=None):
    return SirdLoss.apply(theta, batch, obs, kind, ckpt_interval)
