"""torch.autograd binding of the pathwise gradient (argument marshalling only).

``pathwise_functional(u, ctx, M, records)`` returns J_T of the trajectories
replayed with the jump records held fixed (``tk_grad_pathwise``) as a 0-d
tensor whose backward yields dJ_T/du.  The library computes J_T and the
gradient in one call; the gradient is kept for the backward pass.

A tensor on the GPU goes through the device-pointer entry points
(``tk_set_pulses_dev``, ``tk_grad_pathwise_dev``) on torch's current stream:
pulses, J_T and the gradient stay in device memory.  A CPU tensor goes
through the host-pointer calls.
"""

from __future__ import annotations

import numpy as np
import torch

from .trajkrotov import Context


def _device_shape_inputs(ctx: Context, device: torch.device):
    """S and lambda of the context as float64 tensors on `device` (cached)."""
    cache = getattr(ctx, "_dev_inputs", None)
    if cache is None or cache[0] != device:
        S = None if ctx.S is None else torch.as_tensor(
            np.asarray(ctx.S, dtype=np.float64).reshape(ctx.n_ctrl, -1), device=device)
        lam = None if ctx.lam is None else torch.as_tensor(
            np.asarray(ctx.lam, dtype=np.float64), device=device)
        cache = (device, S, lam)
        ctx._dev_inputs = cache
    return cache[1], cache[2]


class PathwiseFunctional(torch.autograd.Function):
    @staticmethod
    def forward(fctx, u: torch.Tensor, ctx: Context, M: int, records: np.ndarray):
        if u.is_cuda:
            ud = u.detach().to(torch.float64).contiguous()
            S, lam = _device_shape_inputs(ctx, u.device)
            stream = torch.cuda.current_stream(u.device).cuda_stream
            ctx.set_pulses_dev(ud.shape[-1], ctx.T, ud.data_ptr(),
                               0 if S is None else S.data_ptr(),
                               0 if lam is None else lam.data_ptr(), stream)
            J = torch.empty((), dtype=torch.float64, device=u.device)
            g = torch.empty((ctx.n_ctrl, ud.shape[-1]), dtype=torch.float64, device=u.device)
            ctx.grad_pathwise_dev(M, records, J.data_ptr(), 0, g.data_ptr(), stream)
            fctx.save_for_backward(g.to(u.dtype))
            return J.to(u.dtype)
        u_np = u.detach().to("cpu", torch.float64).numpy()
        ctx.set_pulses(u_np, ctx.T, ctx.S, ctx.lam)
        J, _tau, g = ctx.grad_pathwise(M, records)
        fctx.save_for_backward(torch.from_numpy(g).to(dtype=u.dtype))
        return torch.tensor(J, dtype=u.dtype)

    @staticmethod
    def backward(fctx, grad_out):
        (g,) = fctx.saved_tensors
        return grad_out * g, None, None, None


def pathwise_functional(u: torch.Tensor, ctx: Context, M: int, records: np.ndarray) -> torch.Tensor:
    """J_T(u) along the fixed jump record, differentiable with respect to u [n_ctrl, nt]."""
    return PathwiseFunctional.apply(u, ctx, M, records)
