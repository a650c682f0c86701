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
        # outputs the loss does not use arrive as None (no zero tensors made)
        ctx.set_materialize_grads(False)
        M = out32[0:1]
        E = out32[1:1 + d]
        C = out32[1 + d:]
        return M, E, C

    @staticmethod
    def backward(ctx, gM, gE, gC):
        (out64,) = ctx.saved_tensors
        d = len(ctx.shape)
        dev = out64.device
        if gM is None and gE is None and gC is None:
            return None, None
        # the partials [gM, gE, gC] in the layout of the moments, zero where
        # the loss does not depend on an output
        n = api.n_moments(d, ctx.cov)
        given = [(0, gM), (1, gE)] + ([(1 + d, gC)] if ctx.cov else [])
        given = [(o, g) for o, g in given if g is not None]
        if len(given) == 1 and given[0][1].numel() == n:
            gmom = given[0][1].reshape(-1).to(torch.float32)
        else:
            gmom = torch.zeros(n, dtype=torch.float32, device=dev)
            for o, g in given:
                gmom[o:o + g.numel()] = g.reshape(-1)
        g = api.moments_adj(ctx.shape, out64, gmom, cov=ctx.cov, device=dev)
        return g, None


def pad_embed(x, shape):
    return PadEmbed.apply(x, tuple(shape))


def mul(a, b):
    return Mul.apply(a, b)


def moments(p, cov=False):
    return Moments.apply(p, cov)


class CapturedStep:
    """A training-style step -- the forward pass of `loss_fn(*leaves)` and
    its backward -- captured once as ONE hipGraph over the given leaf
    tensors themselves, then replayed.  Unlike per-callable graph wrappers,
    nothing is copied into static inputs on a replay: the leaves are the
    graph's inputs (write new values into them in place between replays)
    and every replay leaves the gradients in their ``.grad`` tensors and the
    loss in ``self.loss``.  The gradients are recomputed, not accumulated,
    by each replay.  Warm-up runs (on a side stream, as graph capture needs)
    plan every kernel and allocate the library's workspaces before capture.
    """

    def __init__(self, loss_fn, leaves, warmup=3):
        self.leaves = list(leaves)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(warmup):
                for t in self.leaves:
                    t.grad = None
                loss_fn(*self.leaves).backward()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        for t in self.leaves:
            t.grad = None
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.loss = loss_fn(*self.leaves)
            self.loss.backward()

    def replay(self):
        self.graph.replay()
        return self.loss

