"""Differentiable dequantization + inverse DCT and the decoder-side scale refit.

`DequantIDCT` is a torch.autograd.Function whose forward is
fptc_dequant_idct and whose backward is fptc_dequant_idct_backward: gradients
of any loss on the reconstruction with respect to the per-stream, per-zone
reconstruction scales gamma (FP64 accumulation) and, on request, the
dequantized coefficients.  The decoded symbols are fixed inputs.  `refit`
runs Adam on gamma against the batch MSE to the original signal.
"""
from __future__ import annotations

import torch

from . import fptc as F
from .codec import Decoder


class DequantIDCT(torch.autograd.Function):
    """x = dequant_idct(symbols; gamma).  decoder must hold decoded symbols
    (Decoder.plan() + Decoder.decode() done)."""

    @staticmethod
    def forward(ctx, gamma: torch.Tensor, decoder: Decoder, precision: str = "fp32"):
        d = decoder
        g = gamma.detach().to(torch.float32).contiguous()
        out = torch.empty(max(1, d.batch.n_samples), dtype=torch.float32, device=gamma.device)
        F.fptc_dequant_idct(d.batch.c, d.codec.c, d.lc, d.ws, d.symbols, g, precision, out)
        ctx.decoder = d
        ctx.gamma_dtype = gamma.dtype
        return out[: d.batch.n_samples]

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        d = ctx.decoder
        go = grad_out.to(torch.float32).contiguous()
        gg = torch.empty((d.batch.n_streams, 3), dtype=torch.float64, device=go.device)
        F.fptc_dequant_idct_backward(d.batch.c, d.codec.c, d.lc, d.ws, d.symbols, go, None, gg)
        return gg.to(ctx.gamma_dtype), None, None


def coefficient_grad(decoder: Decoder, grad_out: torch.Tensor) -> torch.Tensor:
    """dL/dchat for every decoded coefficient (window-major per stream)."""
    d = decoder
    gc = torch.empty(max(1, d.batch.n_symbols), dtype=torch.float32, device=grad_out.device)
    F.fptc_dequant_idct_backward(d.batch.c, d.codec.c, d.lc, d.ws, d.symbols,
                                 grad_out.to(torch.float32).contiguous(), gc, None)
    return gc[: d.batch.n_symbols]


def mse(xhat: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """Global mean squared error over every sample of the batch."""
    return torch.mean((xhat - x) ** 2)


def refit(decoder: Decoder, x: torch.Tensor, steps: int = 20, lr: float = 1e-2, betas=(0.9, 0.999),
          eps: float = 1e-8, precision: str = "fp32"):
    """Adam on the per-stream zone scales (start 1) against MSE(decoded, x).
    Returns (gamma [n, 3] float64, losses: the loss before each step and after
    the last)."""
    n = decoder.batch.n_streams
    gamma = torch.ones((n, 3), dtype=torch.float64, device=x.device, requires_grad=True)
    opt = torch.optim.Adam([gamma], lr=lr, betas=betas, eps=eps)
    losses = []
    for _ in range(steps):
        opt.zero_grad(set_to_none=True)
        loss = mse(DequantIDCT.apply(gamma, decoder, precision), x)
        loss.backward()
        losses.append(float(loss.detach()))
        opt.step()
    with torch.no_grad():
        losses.append(float(mse(DequantIDCT.apply(gamma, decoder, precision), x)))
    return gamma.detach(), losses
