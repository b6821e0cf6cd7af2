"""Differentiable projected GEMM: torch.autograd.Function over proj_gemm_save and
proj_gemm_backward_saved.

Forward: R = A Q_{r,K} B (paper Sec. III-A/B), keeping the projections of
its pack step.  Backward (hand-written, in the library's kernels, on those
kept projections): dA = dR (D_N B)_r^T C_N^T and dB = D_N^T (A C_N)_r^T dR,
each one reduced contraction over r * ceil(K / L) projected indices followed
by a synthesis over the groups.  With an orthonormal basis (DCT-II, Haar)
C_N = D_N^T = P, so dA = dR B^T P P^T: the gradient of A is the exact gradient
projected onto the same subspace.
"""
from __future__ import annotations

import torch

from . import projgemm as pg

__all__ = ["ProjGemmFn", "proj_matmul", "ProjLinear"]


class ProjGemmFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, r: int, basis: pg.Basis, prec: str = "bf16"):
        dt = torch.float64 if prec == "f64" else torch.float32
        A_ = A.to(dt).contiguous()
        B_ = B.to(dt).contiguous()
        # the pack step keeps its plain projections A C_N and D_N B, so the
        # backward contracts against them instead of projecting A and B again
        R, saved = pg.gemm_save(A_, B_, r, basis, prec=prec)
        ctx.save_for_backward(saved)
        ctx.r, ctx.basis, ctx.prec = r, basis, prec
        ctx.shape = (A_.shape[0], B_.shape[1], A_.shape[1])
        ctx.in_dtypes = (A.dtype, B.dtype)
        return R.to(A.dtype) if A.dtype != dt else R

    @staticmethod
    def backward(ctx, dR):
        (saved,) = ctx.saved_tensors
        need_a, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_a or need_b):
            return None, None, None, None, None
        dt = torch.float64 if ctx.prec == "f64" else torch.float32
        dR_ = dR.to(dt).contiguous()
        M, W, K = ctx.shape
        dA, dB = pg.gemm_backward_saved(saved, dR_, ctx.r, ctx.basis, M, W, K, prec=ctx.prec, need_dA=need_a,
                                        need_dB=need_b, dtype=dt)
        if dA is not None:
            dA = dA.to(ctx.in_dtypes[0])
        if dB is not None:
            dB = dB.to(ctx.in_dtypes[1])
        return dA, dB, None, None, None


def proj_matmul(A, B, r: int, basis: pg.Basis, prec: str = "bf16"):
    """A Q_{r,K} B with gradients through the projected backward."""
    return ProjGemmFn.apply(A, B, r, basis, prec)


class ProjLinear(torch.nn.Module):
    """y = x Q_{r,in} W: a bias-free linear layer whose contraction over the
    input features runs on the first r projections of each group of L
    features (weight stored in x in_features x out_features)."""

    def __init__(self, weight: torch.Tensor, r: int, basis: pg.Basis, prec: str = "bf16"):
        super().__init__()
        self.weight = torch.nn.Parameter(weight)
        self.r, self.basis, self.prec = r, basis, prec

    def forward(self, x):
        return proj_matmul(x, self.weight, self.r, self.basis, self.prec)
