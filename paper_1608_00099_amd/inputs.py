"""Seeded synthetic workloads (shapes and values), shared by the tests, the
benchmark and the CPU baseline.  Recipes only: nothing here computes any
part of the co-iteration itself.

The paper's workloads are synthetic shapes (Section 3); these generators
draw tensors of the same kind at the sizes of the five benchmark
configurations:
  cfg1  plain pad-embed, d=3: (48,40,36) -> (64,64,64), values U[0,1)
  cfg2  run-time dimension sweep d=2..8, ~2^26 elements per tensor:
        pad-embed into a shape enlarged by 1..16 per axis, and
        x += y*z over the intersection of three shapes
  cfg3  PMF moments, d=6, (16,)*6, Gamma(0.5,1) normalised to sum 1
  cfg4  4096 ragged (x, y) pairs, x zero-padded to s_x + s_y - 1
  cfg5  pad (24,)^5 -> (32,)^5, product with a (28,30,32,26,32) weight,
        E-based loss
Seeds: numpy PCG64 seeded with 1608 + config index (1..5); every tensor
draws from its own SeedSequence child.
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 1608


def seed_seq(cfg: int, *path: int) -> np.random.SeedSequence:
    return np.random.SeedSequence([SEED_BASE + cfg] + [int(p) for p in path])


def rng(cfg: int, *path: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed_seq(cfg, *path)))


def _prod(s):
    p = 1
    for v in s:
        p *= int(v)
    return p


# ---------------------------------------------------------------------------
# cfg1
# ---------------------------------------------------------------------------

CFG1_SRC = (48, 40, 36)
CFG1_DST = (64, 64, 64)


def cfg1_values() -> np.ndarray:
    return rng(1, 0).random(CFG1_SRC, dtype=np.float32)


# ---------------------------------------------------------------------------
# cfg2: shapes with ~2^target elements for a run-time dimension d
# ---------------------------------------------------------------------------

def shape_rule(g: np.random.Generator, d: int, log2_target: float = 26.0):
    """Axes drawn uniformly in [2, 64], then rescaled (at most 6 times) until
    the element count is within a factor sqrt(2) of 2^target.  For d <= 4,
    64^d < 2^26, so the [2, 64] bound is dropped there; for d >= 5 it is
    kept."""
    u = [int(v) for v in g.integers(2, 65, size=d)]
    for _ in range(6):
        lp = math.log2(_prod(u))
        if abs(lp - log2_target) < 0.5:
            break
        f = (2.0 ** log2_target / _prod(u)) ** (1.0 / d)
        u = [max(2, int(round(v * f))) for v in u]
        if d >= 5:
            u = [min(64, v) for v in u]
    return tuple(u)


def _capped_pad(g: np.random.Generator, base, lo: int, hi: int, cap: int):
    """Per-axis enlargement delta ~ U{lo..hi}; while the enlarged shape has
    more than `cap` elements and some delta exceeds 1, the largest delta
    (lowest axis on ties) shrinks by one."""
    delta = [int(v) for v in g.integers(lo, hi + 1, size=len(base))]
    while _prod([b + e for b, e in zip(base, delta)]) > cap and max(delta) > 1:
        i = max(range(len(delta)), key=lambda k: (delta[k], -k))
        delta[i] -= 1
    return tuple(b + e for b, e in zip(base, delta))


def cfg2_pad_shapes(d: int, log2_target: float = 26.0):
    """(src_shape, dst_shape) of the pad-embed at dimension d."""
    g = rng(2, 0, d)
    src = shape_rule(g, d, log2_target)
    dst = _capped_pad(g, src, 1, 16, int(2 ** (log2_target + 2)))
    return src, dst


def cfg2_inter_shapes(d: int, log2_target: float = 26.0):
    """(x_shape, y_shape, z_shape) of x += y*z: x is the counter (and the
    intersection), y and z extend it by 0..16 per axis."""
    g = rng(2, 1, d)
    x = shape_rule(g, d, log2_target)
    cap = int(2 ** (log2_target + 2))
    y = _capped_pad(g, x, 0, 16, cap)
    z = _capped_pad(g, x, 0, 16, cap)
    return x, y, z


def cfg2_inter_literal_shapes(d: int, log2_target: float = 26.0):
    """The literal reading: three independent draws; the counter is their
    elementwise minimum."""
    g = rng(2, 2, d)
    return tuple(shape_rule(g, d, log2_target) for _ in range(3))


def uniform(cfg: int, shape, *path) -> np.ndarray:
    return rng(cfg, *path).random(tuple(shape), dtype=np.float32)


def uniform_torch(shape, seed: int, device):
    """U[0,1) float32 drawn on the device by torch's seeded generator (used
    for the benchmark-scale tensors, where host generation would dominate)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    return torch.rand(tuple(shape), generator=gen, dtype=torch.float32, device=device)


# ---------------------------------------------------------------------------
# Benchmark 1 of the paper (Section 3): crop of a (2^10, 2^9, 2^8) tensor to
# its leading (2^9, 2^9, 2^5) block
# ---------------------------------------------------------------------------

PAPER_B1_BIG = (1 << 10, 1 << 9, 1 << 8)
PAPER_B1_SMALL = (1 << 9, 1 << 9, 1 << 5)


def paper_b1_values(dtype=np.float64) -> np.ndarray:
    """U[0,1) source of the crop in float32 or float64 (the paper's runs use
    float64)."""
    dt = np.dtype(dtype)
    return rng(6, 0, dt.itemsize).random(PAPER_B1_BIG, dtype=dt)


# ---------------------------------------------------------------------------
# cfg3
# ---------------------------------------------------------------------------

CFG3_SHAPE = (16,) * 6


def cfg3_values(shape=CFG3_SHAPE) -> np.ndarray:
    g = rng(3, 0).gamma(0.5, 1.0, size=shape)
    return (g / g.sum()).astype(np.float32)


# ---------------------------------------------------------------------------
# cfg4: ragged pairs for FFT-convolution padding
# ---------------------------------------------------------------------------

def cfg4_shapes(n_pairs: int = 4096, cap: int = 2 ** 18, max_axis: int = 64):
    """[(s_x, s_y)]: d ~ U{1..6}, axes ~ U{1..max_axis}; while the padded
    shape s_x + s_y - 1 exceeds `cap` elements, both axes of the largest
    padded axis (lowest on ties) are halved (rounding up)."""
    g = rng(4, 0)
    out = []
    for _ in range(n_pairs):
        d = int(g.integers(1, 7))
        sx = [int(v) for v in g.integers(1, max_axis + 1, size=d)]
        sy = [int(v) for v in g.integers(1, max_axis + 1, size=d)]
        while _prod([a + b - 1 for a, b in zip(sx, sy)]) > cap:
            i = max(range(d), key=lambda k: (sx[k] + sy[k] - 1, -k))
            sx[i] = (sx[i] + 1) // 2
            sy[i] = (sy[i] + 1) // 2
        out.append((tuple(sx), tuple(sy)))
    return out


def cfg4_values(shapes) -> list:
    g = rng(4, 1)
    return [g.standard_normal(sx).astype(np.float32) for sx, _ in shapes]


def padded_shape(sx, sy):
    """The full linear-convolution shape s_x + s_y - 1 (Algorithm 14's result
    shape)."""
    return tuple(a + b - 1 for a, b in zip(sx, sy))


# ---------------------------------------------------------------------------
# cfg5: the differentiable pipeline
# ---------------------------------------------------------------------------

CFG5_X = (24,) * 5
CFG5_P = (32,) * 5
CFG5_W = (28, 30, 32, 26, 32)


def cfg5_values(xs=CFG5_X, ws=CFG5_W):
    x = rng(5, 0).random(xs, dtype=np.float32)
    w = rng(5, 1).random(ws, dtype=np.float32)
    lam = rng(5, 2).standard_normal(len(xs))
    return x, w, lam
