"""Pins for the oracle's inner product (benchmark 2), benchmark 3's update,
marginalization, the nonzero bounding box and the naive convolution
(Algorithms 14 and 15): each checked against something other than the
oracle itself -- exact integer arithmetic in numpy, correctly rounded sums
(math.fsum) with the sequential-summation error bound, numpy/scipy library
routines, closed forms, and brute force on tiny inputs."""
import itertools
import math

import numpy as np
import pytest
import scipy.signal

import oracle


def _window(parent, base, counter):
    """The numpy view of an operand window: the base decoded in the
    parent's shape gives the window start."""
    start = np.unravel_index(base, parent.shape) if parent.size else (0,) * parent.ndim
    sl = tuple(slice(int(s), int(s) + int(c)) for s, c in zip(start, counter))
    return parent[sl]


# ---------------------------------------------------------------------------
# Inner product
# ---------------------------------------------------------------------------

def test_dot_all_ones_counts_the_shared_tuples():
    a = np.ones((6, 5, 4), np.float32)
    b = np.ones((3, 7, 9), np.float32)
    assert oracle.dot((3, 5, 4), [a, b], [a.shape, b.shape]) == 3 * 5 * 4


def test_dot_integer_values_exact_against_numpy():
    rng = np.random.default_rng(1)
    a = rng.integers(-3, 4, size=(9, 8, 7)).astype(np.float32)
    b = rng.integers(-3, 4, size=(6, 10, 5)).astype(np.float32)
    counter = (6, 8, 5)
    want = int(np.sum(a[:6, :8, :5].astype(np.int64) * b[:6, :8, :5].astype(np.int64)))
    assert oracle.dot(counter, [a, b], [a.shape, b.shape]) == want


@pytest.mark.parametrize("f64", [False, True])
def test_dot_within_sequential_bound_of_exact_sum(f64):
    rng = np.random.default_rng(2)
    dt = np.float64 if f64 else np.float32
    a = rng.standard_normal((17, 33)).astype(dt)
    b = rng.standard_normal((20, 31)).astype(dt)
    counter = (17, 31)
    prods = (a[:, :31].astype(np.float64) * b[:17, :].astype(np.float64)).ravel()
    exact = math.fsum(prods.tolist())
    n = prods.size
    bound = n * np.finfo(np.float64).eps * float(np.sum(np.abs(prods)))
    got = oracle.dot(counter, [a, b], [a.shape, b.shape])
    assert abs(got - exact) <= bound
    if not f64:
        # float32 products are exact in double: a transposed or shifted
        # operand changes the exact sum far beyond the bound
        wrong = math.fsum((a[:, :31].astype(np.float64) * b[3:20, :].astype(np.float64)).ravel().tolist())
        assert abs(wrong - exact) > 100 * bound


def test_dot_windows_and_three_operands():
    rng = np.random.default_rng(3)
    pa, pb, pc = (9, 10, 11), (8, 12, 9), (7, 7, 13)
    a = rng.integers(-2, 3, size=pa).astype(np.float32)
    b = rng.integers(-2, 3, size=pb).astype(np.float32)
    c = rng.integers(-2, 3, size=pc).astype(np.float32)
    counter = (4, 5, 6)
    ba = int(np.ravel_multi_index((2, 3, 4), pa))
    bb = int(np.ravel_multi_index((1, 6, 0), pb))
    bc = int(np.ravel_multi_index((3, 1, 5), pc))
    want = int(np.sum(_window(a, ba, counter).astype(np.int64) * _window(b, bb, counter).astype(np.int64)
                      * _window(c, bc, counter).astype(np.int64)))
    got = oracle.dot(counter, [a, b, c], [pa, pb, pc], [ba, bb, bc])
    assert got == want


def test_dot_degenerate():
    a = np.array(2.5, np.float32).reshape(())
    b = np.array(-4.0, np.float32).reshape(())
    assert oracle.dot((), [a, b], [(), ()]) == -10.0
    z = np.ones((3, 4), np.float32)
    assert oracle.dot((3, 0), [z, z], [(3, 4), (3, 4)]) == 0.0


# ---------------------------------------------------------------------------
# Benchmark 3's update
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_xpyx_mz_bit_exact_against_numpy(dt):
    rng = np.random.default_rng(4)
    xs, ys, zs = (13, 8, 5), (20, 9, 7), (15, 8, 9)
    x = rng.standard_normal(xs).astype(dt)
    y = rng.standard_normal(ys).astype(dt)
    z = rng.standard_normal(zs).astype(dt)
    yv, zv = y[:13, :8, :5], z[:13, :8, :5]
    want = (x + yv * x) - zv            # numpy: one rounding per operation
    got = x.copy()
    oracle.xpyx_mz(xs, got, xs, y, ys, z, zs)
    assert got.tobytes() == want.astype(dt).tobytes()


def test_xpyx_mz_is_not_fused():
    e = np.float32(2.0 ** -12)
    x = np.array([1 + e], np.float32)
    y = np.array([-(1 + e)], np.float32)
    z = np.array([0.0], np.float32)
    got = x.copy()
    oracle.xpyx_mz((1,), got, (1,), y, (1,), z, (1,))
    # y*x = -(1 + 2^-11 + 2^-24) rounds (tie to even) to -(1 + 2^-11); a
    # fused multiply-add would keep the 2^-24
    assert got[0] == np.float32(-(2.0 ** -12))


def test_xpyx_mz_special_values_and_windows():
    x = np.array([np.inf, -0.0, 1e-45, np.nan, 3.0, 2.0], np.float32)
    y = np.array([0.0, 1.0, 1.0, 1.0, -1.0, 0.5], np.float32)
    z = np.array([0.0, 0.0, -1e-45, 0.0, 1.0, np.inf], np.float32)
    with np.errstate(all="ignore"):
        want = (x + y * x) - z
    got = x.copy()
    oracle.xpyx_mz((6,), got, (6,), y, (6,), z, (6,))
    assert got.tobytes() == want.tobytes()
    # windows with bases in all three operands
    rng = np.random.default_rng(5)
    px, py, pz = (10, 9), (12, 14), (9, 20)
    c = (4, 6)
    bx, by, bz = 2 * 9 + 3, 5 * 14 + 7, 1 * 20 + 11
    X = rng.standard_normal(px).astype(np.float32)
    Y = rng.standard_normal(py).astype(np.float32)
    Z = rng.standard_normal(pz).astype(np.float32)
    want = X.copy()
    wx = _window(want, bx, c)
    wx[...] = (wx + _window(Y, by, c) * wx) - _window(Z, bz, c)
    got = X.copy()
    oracle.xpyx_mz(c, got, px, Y, py, Z, pz, bx, by, bz)
    assert got.tobytes() == want.tobytes()


# ---------------------------------------------------------------------------
# Marginalization
# ---------------------------------------------------------------------------

def test_marginal_integer_values_exact_against_numpy():
    rng = np.random.default_rng(6)
    a = rng.integers(0, 5, size=(5, 6, 7, 4)).astype(np.float32)
    b = rng.integers(0, 5, size=(7, 6, 9, 4)).astype(np.float32)
    counter = (5, 6, 7, 4)
    prod = a.astype(np.int64) * b[:5, :, :7, :].astype(np.int64)
    for keep in itertools.product([0, 1], repeat=4):
        axes = tuple(i for i in range(4) if not keep[i])
        want = prod.sum(axis=axes) if axes else prod
        got = oracle.marginal(counter, keep, [a, b], [a.shape, b.shape])
        assert got.shape == np.shape(want)
        assert np.array_equal(got, np.asarray(want, dtype=np.float64)), keep


def test_marginal_closed_forms():
    ones = np.ones((3, 4, 5), np.float32)
    got = oracle.marginal((3, 4, 5), [0, 1, 0], [ones], [(3, 4, 5)])
    assert np.array_equal(got, np.full((4,), 15.0))
    # nothing kept: the inner product
    rng = np.random.default_rng(7)
    a = rng.random((6, 7)).astype(np.float32)
    b = rng.random((6, 7)).astype(np.float32)
    m = oracle.marginal((6, 7), [0, 0], [a, b], [(6, 7), (6, 7)])
    assert m.shape == () and float(m) == oracle.dot((6, 7), [a, b], [(6, 7), (6, 7)])
    # everything kept: the element-wise product, exact in double
    m = oracle.marginal((6, 7), [1, 1], [a, b], [(6, 7), (6, 7)])
    assert np.array_equal(m, a.astype(np.float64) * b.astype(np.float64))


def test_marginal_random_within_bound():
    rng = np.random.default_rng(8)
    a = rng.standard_normal((9, 11, 13)).astype(np.float32)
    got = oracle.marginal((9, 11, 13), [1, 0, 1], [a], [a.shape])
    want = a.astype(np.float64).sum(axis=1)
    bound = 11 * np.finfo(np.float64).eps * np.abs(a.astype(np.float64)).sum(axis=1)
    assert np.all(np.abs(got - want) <= 2 * bound)


# ---------------------------------------------------------------------------
# Nonzero bounding box
# ---------------------------------------------------------------------------

def _np_bbox(mask):
    nz = np.nonzero(mask)
    if nz[0].size == 0:
        return np.full((mask.ndim, 2), -1, np.int64)
    return np.array([[int(v.min()), int(v.max())] for v in nz], np.int64)


def test_bbox_against_numpy_nonzero():
    rng = np.random.default_rng(9)
    a = (rng.random((12, 15, 9)) < 0.02).astype(np.float32) * rng.standard_normal((12, 15, 9)).astype(np.float32)
    b = (rng.random((14, 15, 11)) < 0.5).astype(np.float32) * -2.0
    counter = (12, 15, 9)
    mask = (a != 0) & (b[:12, :, :9] != 0)
    got = oracle.bbox(counter, [a, b], [a.shape, b.shape])
    assert np.array_equal(got, _np_bbox(mask))


def test_bbox_empty_single_nan_and_negative_zero():
    z = np.zeros((4, 5), np.float32)
    assert np.array_equal(oracle.bbox((4, 5), [z], [(4, 5)]), np.full((2, 2), -1))
    z[2, 3] = np.nan
    assert np.array_equal(oracle.bbox((4, 5), [z], [(4, 5)]), [[2, 2], [3, 3]])
    z[2, 3] = -0.0
    z[0, 4] = -1e-45
    z[3, 0] = -7.0
    assert np.array_equal(oracle.bbox((4, 5), [z], [(4, 5)]), [[0, 3], [0, 4]])


def test_bbox_window():
    p = np.zeros((10, 10), np.float64)
    p[4, 7] = 1.0
    p[6, 5] = 2.0
    base = 3 * 10 + 4            # window starting at (3, 4), extents (5, 5)
    got = oracle.bbox((5, 5), [p], [(10, 10)], [base])
    assert np.array_equal(got, [[1, 3], [1, 3]])


# ---------------------------------------------------------------------------
# Naive convolution
# ---------------------------------------------------------------------------

def _brute_conv(l, r):
    """Algorithm 14's loops written out for tiny inputs: every lhs tuple in
    lexicographic order, inside it every rhs tuple."""
    out = np.zeros(tuple(a + b - 1 for a, b in zip(l.shape, r.shape)))
    for t in itertools.product(*[range(s) for s in l.shape]):
        for u in itertools.product(*[range(s) for s in r.shape]):
            v = tuple(a + b for a, b in zip(t, u))
            out[v] = out[v] + l[t] * r[u]
    return out


def test_conv_integer_values_exact_against_scipy():
    rng = np.random.default_rng(10)
    for ls, rs in [((5,), (3,)), ((4, 6), (3, 2)), ((3, 4, 5), (2, 3, 2)), ((256, 8), (256, 8))]:
        l = rng.integers(-4, 5, size=ls).astype(np.float64)
        r = rng.integers(-4, 5, size=rs).astype(np.float64)
        want = scipy.signal.convolve(l, r, method="direct")
        got = oracle.conv(l, r)
        assert got.shape == want.shape and np.array_equal(got, want), (ls, rs)


def test_conv_delta_shifts_and_commutes():
    rng = np.random.default_rng(11)
    r = rng.standard_normal((4, 5, 3))
    delta = np.zeros((2, 3, 2))
    delta[1, 2, 0] = 1.0
    got = oracle.conv(delta, r)
    want = np.zeros((5, 7, 4))
    want[1:5, 2:7, 0:3] = r
    assert np.array_equal(got, want)
    li = rng.integers(-3, 4, size=(6, 4)).astype(np.float64)
    ri = rng.integers(-3, 4, size=(3, 7)).astype(np.float64)
    assert np.array_equal(oracle.conv(li, ri), oracle.conv(ri, li))


def test_conv_brute_force_order_bit_exact():
    rng = np.random.default_rng(12)
    for ls, rs in [((7,), (4,)), ((3, 4), (4, 2)), ((2, 3, 2), (3, 2, 2)), ((), ())]:
        l = rng.standard_normal(ls)
        r = rng.standard_normal(rs)
        got = oracle.conv(np.ascontiguousarray(l), np.ascontiguousarray(r))
        assert got.tobytes() == _brute_conv(l, r).tobytes(), (ls, rs)


def test_conv_random_within_bound_of_scipy():
    rng = np.random.default_rng(13)
    l = rng.standard_normal((40, 6))
    r = rng.standard_normal((30, 5))
    got = oracle.conv(l, r)
    want = scipy.signal.convolve(l, r, method="direct")
    bound = 30 * 5 * np.finfo(np.float64).eps * scipy.signal.convolve(np.abs(l), np.abs(r),
                                                                        method="direct")
    assert np.all(np.abs(got - want) <= 2 * bound)
