"""torch.autograd wrappers over the library's adjoint kernels.

CURLoss(A, I, J, mask)  ->  ||P_Omega(A - C W^+ R)||_F^2  with C = A(:,J),
    R = A(I,:), W = A(I,J) for fixed index sets: the data-fit term of the
    completion problem (Example 4.4) restricted to the observed set.  Its
    forward is one qcur_backward call in masked-loss mode, which returns the
    loss and, when A needs a gradient, dL/dA (kept for the backward pass,
    which only scales it); W^+ is computed inside that call and never
    stored.
CUR(A, I, J)  ->  B = C W^+ R (materialised).  Its backward is the
    vector-Jacobian product of qcur_backward for the incoming gradient of B.

A is a (4, m, n) float64 or float32 tensor on the GPU; forward and backward
run in A's precision with the pseudoinverse in FP64.  rtol and max_rank are
those of qcur_pinv (max_rank = the predefined rank k of Algorithm 1).
"""
from __future__ import annotations

import torch

from . import qcur as Q


def _compute(A):
    if A.dtype == torch.float64:
        return Q.F64
    if A.dtype == torch.float32:
        return Q.F32
    raise TypeError("CUR autograd supports float64 and float32 inputs")


class CURLossFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, I, J, mask, rtol, max_rank):
        _compute(A)
        need = ctx.needs_input_grad[0]
        dA, loss = Q.backward(A.detach(), I, J, mask=mask, rtol=rtol, max_rank=max_rank, want_dA=need)
        ctx.save_for_backward(dA if need else None)
        return loss[0].to(A.dtype)

    @staticmethod
    def backward(ctx, g):
        (dA,) = ctx.saved_tensors
        return g.to(dA.dtype) * dA, None, None, None, None, None


class CURFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, I, J, rtol, max_rank):
        compute = _compute(A)
        C, R, W = Q.gather(A, I, J)
        _, B, _ = Q.approx(None, C, R, W, core=Q.CORE_WPINV, compute=compute, rtol=rtol, max_rank=max_rank,
                           want_B=True)
        ctx.save_for_backward(A, I, J)
        ctx.rtol, ctx.max_rank = rtol, max_rank
        return B.to(A.dtype)

    @staticmethod
    def backward(ctx, gB):
        A, I, J = ctx.saved_tensors
        dA, _ = Q.backward(A, I, J, gB=gB.contiguous().to(A.dtype), rtol=ctx.rtol, max_rank=ctx.max_rank)
        return dA, None, None, None, None


def cur_loss(A, I, J, mask=None, rtol: float = -1.0, max_rank: int = 0):
    """||P_Omega(A - C W^+ R)||_F^2 (mask None = all entries)."""
    return CURLossFn.apply(A, I, J, mask, rtol, max_rank)


def cur(A, I, J, rtol: float = -1.0, max_rank: int = 0):
    """B = C W^+ R for fixed index sets, differentiable in A."""
    return CURFn.apply(A, I, J, rtol, max_rank)
