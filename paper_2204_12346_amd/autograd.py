"""torch.autograd face of the cost: forward = sird_loss, backward =
sird_loss_backward (the discrete adjoint of the RK4 scheme, computed by the
library's HIP kernel with checkpointing every ckpt_interval steps)."""
from __future__ import annotations

import torch

from .core import Batch, sird_loss, sird_loss_backward


class SirdLoss(torch.autograd.Function):
    """loss = SirdLoss.apply(theta, batch, obs, kind, ckpt_interval)

    theta: theta-shaped float64 device tensor of the batch (requires_grad).
    Returns the particle-indexed losses.  backward() gives
    grad_theta = upstream_grad[p] * dL_p/dtheta in the theta layout.
    """

    @staticmethod
    def forward(ctx, theta, batch: Batch, obs, kind="ssre", ckpt_interval=0):
        theta_c = theta.detach().contiguous()
        loss = sird_loss(batch, theta_c, obs, kind)
        ctx.save_for_backward(theta_c, obs)
        ctx.batch = batch
        ctx.kind = kind
        ctx.ckpt_interval = int(ckpt_interval)
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        theta, obs = ctx.saved_tensors
        g = grad_loss.detach().to(torch.float64).contiguous()
        grad, _ = sird_loss_backward(ctx.batch, theta, obs, ctx.kind, grad_loss=g,
                                     ckpt_interval=ctx.ckpt_interval)
        return grad, None, None, None, None


def sird_loss_autograd(theta, batch: Batch, obs, kind="ssre", ckpt_interval=0):
    return SirdLoss.apply(theta, batch, obs, kind, ckpt_interval)
