"""gfx950 (MI355X) library for batched calibration of the SIRD model.

The hot path -- RK4 integration of eq. (SIRD) for every particle of a
particle swarm, fused with the deceased-count cost, plus the swarm update,
the discrete adjoint and refinement -- runs in hand-written HIP kernels
behind the C ABI of ``include/sird.h``; this package is the thin binding.
"""
from . import _lib
from ._lib import LOSS, SirdError
from .core import (CKPT_SEGMENTS, Batch, Graph, LbfgsState, ProblemSpec, PsoParams, Swarm,
                   pso_complete_move, sird_lbfgs_accept, sird_lbfgs_propose,
                   pso_evaluate, pso_gbest, pso_init, pso_step, pso_topk, sird_adam_step,
                   sird_gather, sird_integrate, sird_loss, sird_loss_backward,
                   sird_loss_backward_static, sird_loss_backward_workspace, sird_pso_iterate)

__all__ = [
    "CKPT_SEGMENTS", "Batch", "Graph", "LbfgsState", "ProblemSpec", "PsoParams", "Swarm", "LOSS", "SirdError",
    "pso_complete_move", "pso_evaluate", "pso_gbest", "pso_init", "pso_step", "pso_topk",
    "sird_adam_step", "sird_gather", "sird_integrate", "sird_lbfgs_accept",
    "sird_lbfgs_propose", "sird_loss", "sird_loss_backward", "sird_loss_backward_static",
    "sird_loss_backward_workspace", "sird_pso_iterate",
]
