"""FFT convolution around the co-iteration kernels (the task that motivates
the paper, Sections 1 and 3): zero-pad both operands into a common
FFT-friendly shape (EMBED_FILL, one pass each), transform, multiply,
transform back, and crop the linear-convolution result (COPY, benchmark 1's
crop) out of the padded tensor.

The transforms are the device FFT library's (rocFFT, through torch.fft);
padding and cropping are this library's kernels.  For a ragged batch the
pads and the crops each run as one batched launch (a persistent kernel
over all items, replayed from a captured graph), and the transforms run
per item (their shapes differ)."""
from __future__ import annotations

import torch

from . import api


def good_size(n: int) -> int:
    """The least m >= n whose prime factors are 2, 3 and 5 only (sizes the
    FFT library transforms fastest)."""
    if n <= 1:
        return 1
    m = n
    while True:
        r = m
        for p in (2, 3, 5):
            while r % p == 0:
                r //= p
        if r == 1:
            return m
        m += 1


def conv_shape(sx, sy):
    return tuple(a + b - 1 for a, b in zip(sx, sy))


def fft_conv(x: torch.Tensor, y: torch.Tensor, batch_dims: int = 0) -> torch.Tensor:
    """Linear convolution of x and y over their trailing dimensions (the
    first ``batch_dims`` dimensions are a batch shared by both), via FFT.
    float32 or float64; the result has shape batch + (sx + sy - 1)."""
    if x.dtype != y.dtype or x.dtype not in (torch.float32, torch.float64):
        raise ValueError("fft_conv takes two float32 or two float64 tensors")
    b = tuple(x.shape[:batch_dims])
    if tuple(y.shape[:batch_dims]) != b:
        raise ValueError("batch dimensions differ")
    sx, sy = tuple(x.shape[batch_dims:]), tuple(y.shape[batch_dims:])
    if len(sx) != len(sy):
        raise ValueError("x and y must have the same dimension")
    s = conv_shape(sx, sy)
    n = tuple(good_size(v) for v in s)
    xp = api.pad_embed(x.contiguous(), b + n)
    yp = api.pad_embed(y.contiguous(), b + n)
    dims = tuple(range(batch_dims, batch_dims + len(n)))
    spec = torch.fft.rfftn(xp, dim=dims) * torch.fft.rfftn(yp, dim=dims)
    full = torch.fft.irfftn(spec, s=n, dim=dims).contiguous()
    return api.crop(full, b + s)


class RaggedFFTConv:
    """FFT convolution of a ragged batch of pairs (x_i, y_i) (any dimension,
    any shapes per pair): one batched zero-pad launch for all x_i, one for
    all y_i, per-item transforms, one batched crop launch.  The pad and crop
    batches are planned and captured on the first call and replayed while
    the pairs' shapes repeat."""

    def __init__(self):
        self._pad_x = api.Batch()
        self._pad_y = api.Batch()
        self._crop = api.Batch()

    def close(self):
        for b in (self._pad_x, self._pad_y, self._crop):
            b.close()

    def __call__(self, xs, ys):
        dev = xs[0].device
        dt = xs[0].dtype
        pads_x, pads_y, outs, fulls = [], [], [], []
        for x, y in zip(xs, ys):
            s = conv_shape(x.shape, y.shape)
            n = tuple(good_size(v) for v in s)
            pads_x.append(torch.empty(n, dtype=dt, device=dev))
            pads_y.append(torch.empty(n, dtype=dt, device=dev))
            outs.append(torch.empty(s, dtype=dt, device=dev))
        from . import _lib as L
        eb = xs[0].element_size()
        self._pad_x.apply(L.OP_EMBED_FILL, [[p, x] for p, x in zip(pads_x, xs)], elem_bytes=eb)
        self._pad_y.apply(L.OP_EMBED_FILL, [[p, y] for p, y in zip(pads_y, ys)], elem_bytes=eb)
        for xp, yp in zip(pads_x, pads_y):
            spec = torch.fft.rfftn(xp) * torch.fft.rfftn(yp)
            fulls.append(torch.fft.irfftn(spec, s=tuple(xp.shape)).contiguous())
        # crop: COPY over the default counter, the intersection = the result shape
        self._crop.apply(L.OP_COPY, [[o, f] for o, f in zip(outs, fulls)], elem_bytes=eb)
        return outs
