"""Differentiable y = A L^{-1} b on the fused executor.

Forward: one fused SpTRSV -> SpMV launch.  Backward: one launch of the
adjoint executor, which runs the transposed solve over its own reversed
schedule with c = A^T g computed inside each row:
    lambda = L^{-T} (A^T g),  grad_b = lambda,
    grad_L = -(lambda x^T) restricted to the stored pattern of L.
With ``recompute_x=True`` the forward keeps only b and the backward
re-solves x (activation recomputation instead of storage).  A's values are
treated as constants (no gradient).
"""
from __future__ import annotations

import torch


class TrsvSpmv(torch.autograd.Function):
    @staticmethod
    def forward(ctx, L_val, b, A_val, sched, recompute_x=False):
        from . import trsv_spmv
        x, y = trsv_spmv(sched, L_val, A_val, b)
        ctx.sched = sched
        ctx.recompute_x = bool(recompute_x)
        if recompute_x:
            ctx.save_for_backward(L_val, A_val, b)
        else:
            ctx.save_for_backward(L_val, A_val, x)
        return y

    @staticmethod
    def backward(ctx, gy):
        from . import backward
        L_val, A_val, v = ctx.saved_tensors
        g = gy.contiguous()
        if ctx.recompute_x:
            grad_b, grad_l = backward(ctx.sched, L_val, A_val, g, B=v)
        else:
            grad_b, grad_l = backward(ctx.sched, L_val, A_val, g, X=v)
        return grad_l, grad_b, None, None, None


def trsv_spmv_autograd(L_val, b, A_val, sched, recompute_x=False):
    """y = A L^{-1} b with gradients for L's stored values and b."""
    return TrsvSpmv.apply(L_val, b, A_val, sched, recompute_x)
