"""Differentiable forms: torch.autograd.Functions whose forward and backward
passes are the library's kernels.

  PadEmbed  forward: zero-filled embedding (EMBED_FILL)
            backward: crop-gather (COPY over the source shape)
  Mul       forward: product over the intersection (MUL)
            backward: broadcast-scatter (MUL_ADJ, zero outside the intersection)
  Moments   forward: index-weighted moments (MOMENTS, Algorithm 11)
            backward: index-weighted scatter (MOMENTS_ADJ)
"""
from __future__ import annotations

import torch

from . import api


class PadEmbed(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, shape):
        ctx.src_shape = tuple(x.shape)
        return api.pad_embed(x.contiguous(), tuple(shape))

    @staticmethod
    def backward(ctx, g):
        return api.crop(g.contiguous(), ctx.src_shape), None


class Mul(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, b):
        a = a.contiguous()
        b = b.contiguous()
        ctx.save_for_backward(a, b)
        return api.mul(a, b)

    @staticmethod
    def backward(ctx, g):
        a, b = ctx.saved_tensors
        ga, gb = api.mul_adj(g.contiguous(), a, b)
        return ga, gb


class Moments(torch.autograd.Function):
    """Returns (M, E, C); C is empty unless cov=True (upper triangle).  In a
    pipeline the weights are the previous op's output, so they are loaded
    through the caches (a hint; the results do not depend on it)."""

    @staticmethod
    def forward(ctx, p, cov):
        p = p.contiguous()
        out32, out64 = api.moments(p, cov=cov, cached=True)
        d = p.dim()
        ctx.cov = bool(cov)
        ctx.shape = tuple(p.shape)
        ctx.save_for_backward(out64)
        M = out32[0:1]
        E = out32[1:1 + d]
        C = out32[1 + d:]
        return M, E, C

    @staticmethod
    def backward(ctx, gM, gE, gC):
        (out64,) = ctx.saved_tensors
        d = len(ctx.shape)
        dev = out64.device
        parts = [gM if gM is not None else torch.zeros(1, device=dev),
                 gE if gE is not None else torch.zeros(d, device=dev)]
        if ctx.cov:
            parts.append(gC if gC is not None else torch.zeros(d * (d + 1) // 2, device=dev))
        gmom = torch.cat([p.reshape(-1).to(torch.float32) for p in parts])
        g = api.moments_adj(ctx.shape, out64, gmom, cov=ctx.cov, device=dev)
        return g, None


def pad_embed(x, shape):
    return PadEmbed.apply(x, tuple(shape))


def mul(a, b):
    return Mul.apply(a, b)


def moments(p, cov=False):
    return Moments.apply(p, cov)
