"""torch.autograd binding of the pathwise gradient (argument marshalling only).

``pathwise_functional(u, ctx, M, records)`` returns J_T of the trajectories
replayed with the jump records held fixed (``tk_grad_pathwise``) as a 0-d
tensor whose backward yields dJ_T/du.  The library computes J_T and the
gradient in one call; the gradient is kept for the backward pass.
"""

from __future__ import annotations

import numpy as np
import torch

from .trajkrotov import Context


class PathwiseFunctional(torch.autograd.Function):
    @staticmethod
    def forward(fctx, u: torch.Tensor, ctx: Context, M: int, records: np.ndarray):
        u_np = u.detach().to("cpu", torch.float64).numpy()
        ctx.set_pulses(u_np, ctx.T, ctx.S, ctx.lam)
        J, _tau, g = ctx.grad_pathwise(M, records)
        fctx.save_for_backward(torch.from_numpy(g).to(device=u.device, dtype=u.dtype))
        return torch.tensor(J, dtype=u.dtype, device=u.device)

    @staticmethod
    def backward(fctx, grad_out):
        (g,) = fctx.saved_tensors
        return grad_out * g, None, None, None


def pathwise_functional(u: torch.Tensor, ctx: Context, M: int, records: np.ndarray) -> torch.Tensor:
    """J_T(u) along the fixed jump record, differentiable with respect to u [n_ctrl, nt]."""
    return PathwiseFunctional.apply(u, ctx, M, records)
