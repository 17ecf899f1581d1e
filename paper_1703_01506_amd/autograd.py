"""torch.autograd binding of the masked completion loss of Eq. 1.

    loss = masked_subspace_loss(U, W, omega_ptr, omega_idx, t_vals)
    loss.backward()          # U.grad, W.grad from the library's backward kernel

f(U, W) = 1/2 sum_b sum_{k in Omega_b} (t_bk - U[k, :] W[:, b])^2 over CSR
sampled sets (omega_ptr int64 [B + 1], omega_idx int32 [nnz], t_vals FP32
[nnz]); U is v x r, W is r x B, both FP32 on the GPU.  The forward and the
backward run rpt_masked_loss_fwd / rpt_masked_loss_bwd; the incoming gradient
is applied inside the backward kernel.  The loss is an FP64 scalar tensor.
"""
from __future__ import annotations

import torch

from . import api


class MaskedSubspaceLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, W, omega_ptr, omega_idx, t_vals):
        U = U.contiguous()
        W = W.contiguous()
        loss, resid = api.masked_loss_fwd(U, W, omega_ptr, omega_idx, t_vals)
        ctx.save_for_backward(U, W, omega_ptr, omega_idx, resid)
        return loss.reshape(())

    @staticmethod
    def backward(ctx, grad):
        U, W, omega_ptr, omega_idx, resid = ctx.saved_tensors
        g = grad.detach().reshape(1).to(torch.float64).contiguous()
        dU, dW = api.masked_loss_bwd(U, W, omega_ptr, omega_idx, resid, grad_scale=g)
        return dU, dW, None, None, None


def masked_subspace_loss(U, W, omega_ptr, omega_idx, t_vals):
    return MaskedSubspaceLoss.apply(U, W, omega_ptr, omega_idx, t_vals)
