"""Pins for the oracle's adjoints and the float64 pipeline gradient.

References: central finite differences in float64, and dot-product
(transpose) identities that hold exactly with integer-valued inputs.
"""
import numpy as np
import pytest

import oracle
from oracle import pipeline


def _loss_from_moments(mom, gmom):
    return float(np.dot(mom, gmom))


@pytest.mark.parametrize("cov", [False, True])
def test_moments_adj_matches_finite_differences(cov):
    rng = np.random.default_rng(61)
    shape = (3, 4, 5)
    d = len(shape)
    w = rng.random(shape) + 0.2
    nout = 1 + d + d * (d + 1) // 2
    gmom = rng.standard_normal(nout)
    if not cov:
        gmom[1 + d:] = 0.0
    mom = oracle.moments(shape, [w.reshape(-1)], [shape], cov=True)
    g = np.zeros(shape)
    oracle.moments_adj(shape, g.reshape(-1), shape, mom, gmom, cov=cov)
    h = 1e-6
    flat = w.reshape(-1)
    for k in rng.choice(flat.size, size=20, replace=False):
        wp, wm = flat.copy(), flat.copy()
        wp[k] += h
        wm[k] -= h
        lp = _loss_from_moments(oracle.moments(shape, [wp], [shape]), gmom)
        lm = _loss_from_moments(oracle.moments(shape, [wm], [shape]), gmom)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g.reshape(-1)[k]) <= 1e-6 * max(1.0, abs(fd))


def test_moments_adj_float32_output_is_rounded_float64():
    rng = np.random.default_rng(62)
    shape = (4, 3)
    w = rng.random(shape)
    mom = oracle.moments(shape, [w.reshape(-1)], [shape])
    gmom = rng.standard_normal(mom.size)
    g64 = np.zeros(shape)
    g32 = np.zeros(shape, dtype=np.float32)
    oracle.moments_adj(shape, g64.reshape(-1), shape, mom, gmom)
    oracle.moments_adj(shape, g32.reshape(-1), shape, mom, gmom)
    assert g32.tobytes() == g64.astype(np.float32).tobytes()


def test_embed_crop_transpose_identity():
    rng = np.random.default_rng(63)
    xs, ps = (3, 4, 2), (5, 6, 4)
    x = rng.integers(-9, 9, size=xs).astype(np.float64)
    y = rng.integers(-9, 9, size=ps).astype(np.float64)
    ex = np.zeros(ps)
    oracle.copy(xs, ex.reshape(-1), ps, x.reshape(-1), xs)
    cy = np.zeros(xs)
    oracle.copy(xs, cy.reshape(-1), xs, y.reshape(-1), ps)
    assert float((ex * y).sum()) == float((x * cy).sum())


def test_mul_adj_transpose_identity():
    rng = np.random.default_rng(64)
    sa, sb, si = (5, 6, 4), (3, 6, 5), (3, 5, 4)
    a = rng.integers(-5, 5, size=sa).astype(np.float64)
    b = rng.integers(-5, 5, size=sb).astype(np.float64)
    u = rng.integers(-5, 5, size=si).astype(np.float64)
    va = rng.integers(-5, 5, size=sa).astype(np.float64)
    vb = rng.integers(-5, 5, size=sb).astype(np.float64)
    # J_a v = (v * b) over I, J_b v = (a * v) over I
    ja = np.zeros(si)
    oracle.mul(si, ja.reshape(-1), si, va.reshape(-1), sa, b.reshape(-1), sb)
    jb = np.zeros(si)
    oracle.mul(si, jb.reshape(-1), si, a.reshape(-1), sa, vb.reshape(-1), sb)
    ga = np.zeros(sa)
    gb = np.zeros(sb)
    oracle.mul_adj(ga.reshape(-1), sa, gb.reshape(-1), sb, u.reshape(-1), si,
                   a.reshape(-1), b.reshape(-1))
    assert float((ja * u).sum()) == float((va * ga).sum())
    assert float((jb * u).sum()) == float((vb * gb).sum())


def test_pipeline_gradient_matches_finite_differences():
    # The differentiable workload at a reduced size: embed (4,3,5)->(6,5,7),
    # product with a (5,4,6) weight over the intersection, E-based loss.
    rng = np.random.default_rng(65)
    xs, ps, ish = (4, 3, 5), (6, 5, 7), (5, 4, 6)
    x = rng.random(xs)
    w = rng.random(ish)
    lam = rng.standard_normal(len(xs))
    gx, gw = pipeline.gradient(x.reshape(-1), w.reshape(-1), lam, xs, ps, ish)
    for vec, grad, which in ((x, gx, 0), (w, gw, 1)):
        flat = vec.reshape(-1)
        # random unit directions
        for _ in range(4):
            v = rng.standard_normal(flat.size)
            v /= np.linalg.norm(v)
            h = 1e-5
            args_p = [x.reshape(-1), w.reshape(-1)]
            args_m = [x.reshape(-1), w.reshape(-1)]
            args_p[which] = flat + h * v
            args_m[which] = flat - h * v
            fd = (pipeline.loss(*args_p, lam, xs, ps, ish) -
                  pipeline.loss(*args_m, lam, xs, ps, ish)) / (2 * h)
            assert abs(fd - float(np.dot(grad, v))) <= 1e-7 * max(1.0, abs(fd))
        # coordinates
        for k in rng.choice(flat.size, size=8, replace=False):
            h = 1e-4
            e = np.zeros(flat.size)
            e[k] = h
            args_p = [x.reshape(-1), w.reshape(-1)]
            args_m = [x.reshape(-1), w.reshape(-1)]
            args_p[which] = flat + e
            args_m[which] = flat - e
            fd = (pipeline.loss(*args_p, lam, xs, ps, ish) -
                  pipeline.loss(*args_m, lam, xs, ps, ish)) / (2 * h)
            assert abs(fd - grad[k]) <= 1e-6 * max(abs(grad).max(), 1e-12)
