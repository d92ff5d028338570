"""Differentiable dequantization + inverse DCT and the decoder-side scale refit.

`DequantIDCT` is a torch.autograd.Function whose forward is
fptc_dequant_idct and whose backward is fptc_dequant_idct_backward: gradients
of any loss on the reconstruction with respect to the per-stream, per-zone
reconstruction scales gamma (FP64 accumulation) and the coefficients (through
its optional additive coefficient input).  The decoded symbols are fixed
inputs.  `refit`
runs Adam on gamma against the batch MSE to the original signal.
"""
from __future__ import annotations

import numpy as np
import torch

from . import fptc as F
from .codec import Decoder


class DequantIDCT(torch.autograd.Function):
    """x = IDCT(gamma * dequant(symbols) + delta): the decoder's reconstruction
    with per-stream zone scales gamma [n_streams, 3] and an optional additive
    coefficient tensor delta [n_symbols] (window-major per stream, the
    symbols' layout; None = 0).  Its backward is the library's
    dequant+IDCT backward: the gradient of gamma (FP64 sums) and of the
    coefficients (for delta) come from one call.  decoder must hold decoded
    symbols (Decoder.plan() + Decoder.decode() done).  The reconstruction of
    the symbols runs in the library; the delta term, a training-side input,
    is one dense product with the IDCT basis per window."""

    @staticmethod
    def forward(ctx, gamma: torch.Tensor, decoder: Decoder, precision: str = "fp32", delta=None):
        d = decoder
        g = gamma.detach().to(torch.float32).contiguous()
        out = torch.empty(max(1, d.batch.n_samples), dtype=torch.float32, device=gamma.device)
        F.fptc_dequant_idct(d.batch.c, d.codec.c, d.lc, d.ws, d.symbols, g, precision, out)
        out = out[: d.batch.n_samples]
        if delta is not None:
            out = out + idct_coefficients(d, delta.detach())
        ctx.decoder = d
        ctx.gamma_dtype = gamma.dtype
        ctx.delta_dtype = None if delta is None else delta.dtype
        return out

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        d = ctx.decoder
        go = grad_out.to(torch.float32).contiguous()
        gg = torch.empty((d.batch.n_streams, 3), dtype=torch.float64, device=go.device)
        gc = None
        if ctx.delta_dtype is not None and ctx.needs_input_grad[3]:
            gc = torch.empty(max(1, d.batch.n_symbols), dtype=torch.float32, device=go.device)
        F.fptc_dequant_idct_backward(d.batch.c, d.codec.c, d.lc, d.ws, d.symbols, go, gc, gg)
        gdelta = None if gc is None else gc[: d.batch.n_symbols].to(ctx.delta_dtype)
        return gg.to(ctx.gamma_dtype), None, None, gdelta


def window_sample_index(sample_off: np.ndarray, N: int) -> np.ndarray:
    """For each sample of a batch's windows (window-major, N per window,
    streams in order) its index in the output, or -1 past its stream's end."""
    so = np.asarray(sample_off, dtype=np.int64)
    lens = np.diff(so)
    nw = (lens + N - 1) // N
    w_stream = np.repeat(np.arange(lens.shape[0]), nw)  # stream of each window
    w_first = np.repeat(np.cumsum(nw) - nw, nw)         # the stream's first window
    w_rel = np.arange(int(nw.sum())) - w_first          # window within the stream
    pos = (w_rel * N)[:, None] + np.arange(N)[None, :]  # sample within the stream
    return np.where(pos < lens[w_stream][:, None], so[w_stream][:, None] + pos, -1).reshape(-1)


def _window_samples(decoder: Decoder) -> torch.Tensor:
    d = decoder
    m = getattr(d, "_window_samples", None)
    if m is None:
        idx = window_sample_index(d.batch.sample_off_h, d.codec.N)
        m = torch.from_numpy(idx.astype(np.int64)).to(d.out.device)
        d._window_samples = m
    return m


def idct_coefficients(decoder: Decoder, delta: torch.Tensor) -> torch.Tensor:
    """The batch's samples of IDCT(delta) for coefficients delta [n_symbols]
    in the symbols' layout (Section 3.1, orthonormal inverse of the kept bins)."""
    d = decoder
    E = d.codec.E
    X = torch.matmul(delta.to(torch.float32).reshape(-1, E), d.codec.basis.reshape(E, d.codec.N))
    m = _window_samples(d)
    keep = m >= 0
    out = torch.zeros(max(1, d.batch.n_samples), dtype=torch.float32, device=delta.device)
    out[m[keep]] = X.reshape(-1)[keep]
    return out[: d.batch.n_samples]


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
