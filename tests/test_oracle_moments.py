"""Pins for the oracle's index-weighted moments (Algorithm 11, read as the
expected value E[t_i] of a PMF, plus the covariance of t).

References: exact closed forms (delta, uniform), a textbook 1-D
computation for separable PMFs, numpy's weighted ``average`` and ``cov``
(``aweights``, ``bias=True``), exact rational brute force written here with
``fractions``, and invariances (axis permutation, zero padding, window
offsets).
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle


def _unpack(mom, d):
    M = mom[0]
    E = mom[1:1 + d]
    C = np.zeros((d, d))
    p = 1 + d
    for i in range(d):
        for j in range(i, d):
            C[i, j] = C[j, i] = mom[p]
            p += 1
    return M, E, C


@pytest.mark.parametrize("shape,t", [((5,), (3,)), ((4, 7), (3, 0)), ((3, 4, 5, 2), (1, 3, 4, 1)),
                                     ((16,) * 6, (3, 15, 0, 7, 9, 1))])
def test_delta_gives_its_tuple(shape, t):
    p = np.zeros(shape, dtype=np.float32)
    p[t] = 0.375
    M, E, C = _unpack(oracle.moments(shape, [p.reshape(-1)], [shape]), len(shape))
    assert M == 0.375
    assert E.tolist() == list(t)
    assert (C == 0).all()


@pytest.mark.parametrize("shape", [(5,), (4, 9), (3, 6, 2), (16, 16, 16), (2, 3, 4, 5, 6)])
def test_uniform_closed_forms(shape):
    p = np.ones(shape, dtype=np.float32)
    M, E, C = _unpack(oracle.moments(shape, [p.reshape(-1)], [shape]), len(shape))
    s = np.asarray(shape, dtype=np.float64)
    assert M == float(np.prod(s))
    np.testing.assert_allclose(E, (s - 1) / 2, rtol=0, atol=1e-12)
    np.testing.assert_allclose(np.diag(C), (s * s - 1) / 12, rtol=1e-12)
    off = C - np.diag(np.diag(C))
    assert np.abs(off).max() < 1e-12


def test_separable_reduces_to_1d_marginals():
    rng = np.random.default_rng(21)
    shape = (7, 5, 9)
    qs = [rng.random(s) + 0.1 for s in shape]
    p = np.einsum("i,j,k->ijk", *qs)
    M, E, C = _unpack(oracle.moments(shape, [p.reshape(-1)], [shape]), 3)
    for i, q in enumerate(qs):
        k = np.arange(len(q), dtype=np.float64)
        mean = (q * k).sum() / q.sum()
        var = (q * (k - mean) ** 2).sum() / q.sum()
        assert abs(E[i] - mean) < 1e-12
        assert abs(C[i, i] - var) < 1e-12
    off = C - np.diag(np.diag(C))
    assert np.abs(off).max() < 1e-12


@pytest.mark.parametrize("seed", range(5))
def test_matches_numpy_weighted_cov(seed):
    rng = np.random.default_rng(400 + seed)
    d = int(rng.integers(1, 6))
    shape = tuple(int(v) for v in rng.integers(1, 7, size=d))
    p = rng.gamma(0.5, 1.0, size=shape)
    M, E, C = _unpack(oracle.moments(shape, [p.reshape(-1)], [shape]), d)
    idx = np.indices(shape).reshape(d, -1).astype(np.float64)
    w = p.reshape(-1)
    assert abs(M - w.sum()) <= 1e-12 * w.sum()
    np.testing.assert_allclose(E, np.average(idx, axis=1, weights=w), rtol=1e-12, atol=1e-12)
    ref = np.atleast_2d(np.cov(idx, aweights=w, bias=True))
    np.testing.assert_allclose(C, ref, rtol=1e-10, atol=1e-12)


def _exact_moments(shape, w):
    """Exact rational E and C by brute force over all tuples."""
    d = len(shape)
    M = Fraction(0)
    S = [Fraction(0)] * d
    for t in itertools.product(*[range(s) for s in shape]):
        wt = Fraction(int(w[t]))
        M += wt
        for i in range(d):
            S[i] += wt * t[i]
    E = [s / M for s in S]
    C = [[Fraction(0)] * d for _ in range(d)]
    for t in itertools.product(*[range(s) for s in shape]):
        wt = Fraction(int(w[t]))
        for i in range(d):
            for j in range(d):
                C[i][j] += wt * (t[i] - E[i]) * (t[j] - E[j])
    return M, E, [[c / M for c in row] for row in C]


@pytest.mark.parametrize("shape", [(3, 4), (2, 3, 4), (4, 2, 2, 3)])
def test_exact_rational_brute_force(shape):
    rng = np.random.default_rng(sum(shape))
    w = rng.integers(0, 50, size=shape).astype(np.float32)
    M, E, C = _unpack(oracle.moments(shape, [w.reshape(-1)], [shape]), len(shape))
    Mx, Ex, Cx = _exact_moments(shape, w)
    assert M == float(Mx)
    for i in range(len(shape)):
        assert abs(E[i] - float(Ex[i])) <= 1e-14 * max(1.0, abs(float(Ex[i])))
        for j in range(len(shape)):
            assert abs(C[i, j] - float(Cx[i][j])) <= 1e-13 * max(1.0, abs(float(Cx[i][j])))


def test_axis_permutation_permutes_moments():
    rng = np.random.default_rng(33)
    shape = (4, 6, 5)
    p = rng.random(shape)
    perm = (2, 0, 1)
    q = np.ascontiguousarray(np.transpose(p, perm))
    M1, E1, C1 = _unpack(oracle.moments(shape, [p.reshape(-1)], [shape]), 3)
    M2, E2, C2 = _unpack(oracle.moments(q.shape, [q.reshape(-1)], [q.shape]), 3)
    assert abs(M1 - M2) <= 1e-13 * M1
    np.testing.assert_allclose(E2, E1[list(perm)], rtol=1e-12)
    np.testing.assert_allclose(C2, C1[np.ix_(perm, perm)], rtol=1e-10, atol=1e-13)


def test_padding_and_window_offsets():
    rng = np.random.default_rng(34)
    shape, big = (4, 5, 3), (9, 8, 7)
    p = rng.random(shape).astype(np.float32)
    ref = oracle.moments(shape, [p.reshape(-1)], [shape])
    # zero padding at the origin leaves every moment unchanged
    P = np.zeros(big, dtype=np.float32)
    P[:4, :5, :3] = p
    padded = oracle.moments(big, [P.reshape(-1)], [big])
    np.testing.assert_allclose(padded, ref, rtol=1e-12, atol=1e-14)
    # embedding at offset beta shifts E by beta and leaves C unchanged
    beta = (3, 2, 4)
    Q = np.zeros(big, dtype=np.float32)
    Q[3:7, 2:7, 4:7] = p
    shifted = oracle.moments(big, [Q.reshape(-1)], [big])
    np.testing.assert_allclose(shifted[1:4], ref[1:4] + np.asarray(beta), rtol=1e-12)
    np.testing.assert_allclose(shifted[4:], ref[4:], rtol=1e-9, atol=1e-12)
    # ... and a window (base offset) onto Q reproduces the unshifted moments
    base = int(np.ravel_multi_index(beta, big))
    win = oracle.moments(shape, [Q.reshape(-1)], [big], bases=[base])
    np.testing.assert_allclose(win, ref, rtol=1e-12, atol=1e-14)


def test_product_of_operands_is_the_weight():
    # Algorithm 11 weights every tuple by the product of all operands.
    rng = np.random.default_rng(35)
    shape = (3, 4, 5)
    xs, ys, zs = (3, 4, 5), (5, 4, 6), (4, 7, 5)
    x = rng.random(xs)
    y = rng.random(ys)
    z = rng.random(zs)
    three = oracle.moments(shape, [x.reshape(-1), y.reshape(-1), z.reshape(-1)], [xs, ys, zs])
    w = x * y[:3, :4, :5] * z[:3, :4, :5]
    one = oracle.moments(shape, [np.ascontiguousarray(w).reshape(-1)], [shape])
    np.testing.assert_allclose(three, one, rtol=1e-13, atol=1e-15)


def test_first_only_and_zero_mass():
    p = np.zeros((3, 3), dtype=np.float32)
    mom = oracle.moments((3, 3), [p.reshape(-1)], [(3, 3)], cov=False)
    assert mom[0] == 0.0
    assert np.isnan(mom[1:3]).all()       # 0/0: no expected value exists
    assert (mom[3:] == 0).all()           # covariance not requested
