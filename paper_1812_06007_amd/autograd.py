"""torch.autograd functions over the derivative entry points of liburv.

``power_urv(A, G, q)`` returns (U, R, V) of PowerURV (Section 3, eqs. power
and powerqr) started from the fixed matrix G, differentiable with respect to
A through the hand-written adjoint of every QR and product of the chain
(``urv_factor_tape`` / ``urv_factor_backward``).  ``truncation_loss`` is
||A - U(:,:k) R(:k,:) V^T||_F^2, the squared rank-k error of Section 5,
evaluated with its adjoints in the library's kernels.

Every computation runs in liburv.so; torch only holds the tensors and
accumulates the gradients the two functions return.
"""
from __future__ import annotations

import torch

from . import urv


class PowerURVFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, G, q, variant, tape_mode):
        U, R, V, tape = urv.factor_tape(A, G, q, variant, tape_mode)
        ctx.save_for_backward(A, G, U, R, V)
        ctx.tape = tape
        ctx.q, ctx.variant, ctx.tape_mode = q, variant, tape_mode
        return U, R, V

    @staticmethod
    def backward(ctx, dU, dR, dV):
        A, G, U, R, V = ctx.saved_tensors
        dA = urv.factor_backward(A, G, U, R, V, ctx.tape, ctx.q, dU, dR, dV, ctx.variant, ctx.tape_mode)
        return dA, None, None, None, None


def power_urv(A, G, q: int = 2, variant: str = "full", tape_mode: str = "all"):
    """(U, R, V) with A = U R V^T, differentiable in A with G held fixed."""
    return PowerURVFunction.apply(A, G, q, variant, tape_mode)


class TruncationLossFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, U, R, V, k):
        L, dU, dR, dV, dA = urv.truncation_loss(A, U, R, V, k)
        ctx.save_for_backward(dU, dR, dV, dA)
        return L

    @staticmethod
    def backward(ctx, gL):
        dU, dR, dV, dA = ctx.saved_tensors
        if not (gL.numel() == 1 and float(gL) == 1.0):
            dU, dR, dV, dA = (gL.to(t.dtype) * t for t in (dU, dR, dV, dA))
        return dA, dU, dR, dV, None


def truncation_loss(A, U, R, V, k: int):
    """||A - U(:,:k) R(:k,:) V^T||_F^2 (a 0-d float64 tensor), differentiable in A, U, R and V."""
    return TruncationLossFunction.apply(A, U, R, V, k)
