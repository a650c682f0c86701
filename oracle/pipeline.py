"""Differentiable embed -> product -> moments pipeline, in float64
(TEST INFRASTRUCTURE ONLY).

Composes the oracle's own operations:
  P = zero-pad embedding of x (shape xs) into shape ps     (Section 1)
  y = P[t] * w[t] over the intersection I = shape of w     (Section 4, views)
  E = first moments of y over I                            (Algorithm 11)
  L = sum_i lam_i * E_i
and the analytic gradient through the oracle adjoints (moments_adj,
mul_adj, crop).  Everything is float64 so that central finite
differences can check the gradient.
"""
from __future__ import annotations

import numpy as np

from . import copy, moments, moments_adj, mul, mul_adj


def _n(shape):
    return int(np.prod(shape, dtype=np.int64))


def forward(x, w, lam, xs, ps, ish):
    """Returns (L, P, y, mom) with mom = [M, E_0..E_{d-1}, ...]."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    d = len(xs)
    P = np.zeros(_n(ps), dtype=np.float64)
    copy(xs, P, ps, x, xs)
    y = np.zeros(_n(ish), dtype=np.float64)
    mul(ish, y, ish, P, ps, w, ish)
    mom = moments(ish, [y], [ish], cov=False)
    L = float(np.dot(np.asarray(lam, dtype=np.float64), mom[1:1 + d]))
    return L, P, y, mom


def loss(x, w, lam, xs, ps, ish):
    return forward(x, w, lam, xs, ps, ish)[0]


def gradient(x, w, lam, xs, ps, ish):
    """Analytic (gx, gw) through the oracle adjoints."""
    d = len(xs)
    _, P, y, mom = forward(x, w, lam, xs, ps, ish)
    gmom = np.zeros_like(mom)
    gmom[1:1 + d] = np.asarray(lam, dtype=np.float64)
    gy = np.zeros(_n(ish), dtype=np.float64)
    moments_adj(ish, gy, ish, mom, gmom, cov=False)
    gP = np.zeros(_n(ps), dtype=np.float64)
    gw = np.zeros(_n(ish), dtype=np.float64)
    w64 = np.ascontiguousarray(w, dtype=np.float64)
    mul_adj(gP, ps, gw, ish, gy, ish, P, w64)
    gx = np.zeros(_n(xs), dtype=np.float64)
    copy(xs, gx, xs, gP, ps)  # crop: the adjoint of the origin embedding
    return gx, gw
