"""Differentiable Strassen product.

``StrassenMatmul.apply(A, B, levels, mode)`` returns C = A @ B computed by the
Strassen-fused kernels; its backward computes

    dA = dC @ B^T      (m x k)      -- the kernel reads B^T from B as stored
    dB = A^T @ dC      (k x n)      -- the kernel reads A^T from A as stored

with the same kernels and the same number of Strassen levels (the gradient of
the product C = A B of the Introduction's eq. "prime" with alpha = 1, beta = 0).
No transposed copy is made: the transposed-operand path stages each block of
the stored matrix in the direction it is contiguous in memory.

torch is used for device memory only; every flop runs in libstrassen.so.
"""
import torch

from .api import gemm


def _unit_stride(t):
    # the kernels need unit stride along the second dimension; gradients that
    # arrive expanded or transposed are made contiguous first
    return t if (t.dim() == 2 and (t.shape[1] <= 1 or t.stride(1) == 1)) else t.contiguous()


class StrassenMatmul(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, B, levels=1, mode="plain"):
        if A.dim() != 2 or B.dim() != 2 or A.shape[1] != B.shape[0]:
            raise ValueError("expected A (m x k) and B (k x n)")
        if A.dtype != torch.float32 or B.dtype != torch.float32:
            raise TypeError("StrassenMatmul takes fp32 operands (mode 'plain' or 'bf16x3')")
        A = _unit_stride(A)
        B = _unit_stride(B)
        C = torch.empty(A.shape[0], B.shape[1], device=A.device, dtype=torch.float32)
        gemm(A, B, C, alpha=1.0, beta=0.0, levels=levels, mode=mode)
        ctx.save_for_backward(A, B)
        ctx.levels = levels
        ctx.mode = mode
        return C

    @staticmethod
    def backward(ctx, dC):
        A, B = ctx.saved_tensors
        if dC.dtype != torch.float32:
            raise TypeError("expected an fp32 gradient")
        dC = _unit_stride(dC)
        dA = dB = None
        if ctx.needs_input_grad[0]:
            dA = torch.empty(A.shape, device=A.device, dtype=torch.float32)
            gemm(dC, B, dA, alpha=1.0, beta=0.0, levels=ctx.levels, mode=ctx.mode, trans_b=True)
        if ctx.needs_input_grad[1]:
            dB = torch.empty(B.shape, device=B.device, dtype=torch.float32)
            gemm(A, dC, dB, alpha=1.0, beta=0.0, levels=ctx.levels, mode=ctx.mode, trans_a=True)
        return dA, dB, None, None


def strassen_matmul(A, B, levels=1, mode="plain"):
    """Differentiable C = A @ B with `levels` levels of Strassen."""
    return StrassenMatmul.apply(A, B, levels, mode)
