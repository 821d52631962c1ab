"""Differentiation through the SRT with the hand-written matched adjoint.

Alg. 2 is the exact transpose of Alg. 1 (both are built from the same stored
operator entries), so using it as the backward of Alg. 1 gives the true
gradient of any loss of SRT f -- e.g. dL/df = A^T (A f - g) for the
least-squares loss 0.5 ||A f - g||^2 -- rather than the inconsistent
gradients an approximate adjoint gives. Both directions run in the HIP
library; torch only provides memory and streams.
"""
from __future__ import annotations

import torch

from .srt import SRTPlan


class SRTFunction(torch.autograd.Function):
    """y = A f (Alg. 1) with backward grad_f = A^T grad_y (Alg. 2)."""

    @staticmethod
    def forward(ctx, vol: torch.Tensor, plan: SRTPlan) -> torch.Tensor:
        ctx.plan = plan
        return plan.forward(vol.contiguous())

    @staticmethod
    def backward(ctx, grad_y: torch.Tensor):
        return ctx.plan.adjoint(grad_y.contiguous()), None


class SRTAdjointFunction(torch.autograd.Function):
    """f = A^T y (Alg. 2) with backward grad_y = A grad_f (Alg. 1)."""

    @staticmethod
    def forward(ctx, data: torch.Tensor, plan: SRTPlan) -> torch.Tensor:
        ctx.plan = plan
        return plan.adjoint(data.contiguous())

    @staticmethod
    def backward(ctx, grad_f: torch.Tensor):
        return ctx.plan.forward(grad_f.contiguous()), None


def srt(vol: torch.Tensor, plan: SRTPlan) -> torch.Tensor:
    """Differentiable forward: data = SRT(vol)."""
    return SRTFunction.apply(vol, plan)


def srt_adjoint(data: torch.Tensor, plan: SRTPlan) -> torch.Tensor:
    """Differentiable adjoint: vol = SRT^T(data)."""
    return SRTAdjointFunction.apply(data, plan)


def least_squares_loss(vol: torch.Tensor, data: torch.Tensor, plan: SRTPlan) -> torch.Tensor:
    """0.5 * ||SRT vol - data||^2 summed over the batch (reduced in FP64)."""
    r = srt(vol, plan) - data
    return 0.5 * (r.double() * r.double()).sum()
