"""Pins for the oracle's element-moving and element-wise operations.

References used here, none of them the oracle itself: numpy slicing copies
(the numpy form of benchmark 1, Section 3), ``np.pad``, numpy float32
arithmetic (which never fuses a multiply-add), hard-coded nested loops for
d <= 4 (the C-loop form of benchmark 1), and invariants of the zero-pad
embedding (mass, crop-after-embed, special values kept bit for bit).
"""
import numpy as np
import pytest

import oracle


def _rand_shapes(rng, d, lo=1, hi=7, pad_hi=4):
    src = tuple(int(v) for v in rng.integers(lo, hi, size=d))
    dst = tuple(s + int(rng.integers(0, pad_hi)) for s in src)
    return src, dst


def _sl(counter, start=None):
    start = start or (0,) * len(counter)
    return tuple(slice(a, a + c) for a, c in zip(start, counter))


@pytest.mark.parametrize("seed", range(8))
def test_pad_embed_matches_numpy_slicing(seed):
    rng = np.random.default_rng(seed)
    d = int(rng.integers(1, 6))
    src_s, dst_s = _rand_shapes(rng, d)
    src = rng.random(src_s, dtype=np.float32)
    dst = np.zeros(dst_s, dtype=np.float32)
    oracle.copy(src_s, dst.reshape(-1), dst_s, src.reshape(-1), src_s)
    want = np.zeros(dst_s, dtype=np.float32)
    want[_sl(src_s)] = src
    assert want.tobytes() == dst.tobytes()


@pytest.mark.parametrize("seed", range(8))
def test_crop_matches_numpy_slicing(seed):
    # Benchmark 1 (Section 3): x = y[:x0, :x1, ...] for a larger y.
    rng = np.random.default_rng(50 + seed)
    d = int(rng.integers(1, 6))
    x_s, y_s = _rand_shapes(rng, d)
    y = rng.standard_normal(y_s)           # float64 as in the paper
    x = np.full(x_s, np.nan)
    oracle.copy(x_s, x.reshape(-1), x_s, y.reshape(-1), y_s)
    assert np.array(y[_sl(x_s)]).tobytes() == x.tobytes()


def _c_loop_crop(x, y):
    """Hard-coded loops of the benchmark-1 C form for d <= 4."""
    xs, ys = x.shape, y.shape
    xf, yf = x.reshape(-1), y.reshape(-1)
    d = len(xs)
    if d == 1:
        for i in range(xs[0]):
            xf[i] = yf[i]
    elif d == 2:
        for k in range(xs[0]):
            xb, yb = k * xs[1], k * ys[1]
            for i in range(xs[1]):
                xf[xb + i] = yf[yb + i]
    elif d == 3:
        for k in range(xs[0]):
            for j in range(xs[1]):
                xb = (k * xs[1] + j) * xs[2]
                yb = (k * ys[1] + j) * ys[2]
                for i in range(xs[2]):
                    xf[xb + i] = yf[yb + i]
    else:
        for k in range(xs[0]):
            for j in range(xs[1]):
                for m in range(xs[2]):
                    xb = ((k * xs[1] + j) * xs[2] + m) * xs[3]
                    yb = ((k * ys[1] + j) * ys[2] + m) * ys[3]
                    for i in range(xs[3]):
                        xf[xb + i] = yf[yb + i]


@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_crop_matches_hard_coded_loops(d):
    rng = np.random.default_rng(d)
    x_s, y_s = _rand_shapes(rng, d, lo=2, hi=6)
    y = rng.random(y_s, dtype=np.float32)
    x1 = np.zeros(x_s, dtype=np.float32)
    x2 = np.zeros(x_s, dtype=np.float32)
    _c_loop_crop(x1, y)
    oracle.copy(x_s, x2.reshape(-1), x_s, y.reshape(-1), y_s)
    assert x1.tobytes() == x2.tobytes()


def test_copy_between_windows_with_bases():
    rng = np.random.default_rng(3)
    parent_a, parent_b = (7, 8, 9), (5, 9, 6)
    counter = (3, 4, 5)
    sa, sb = (2, 3, 1), (1, 0, 1)
    a = np.zeros(parent_a, dtype=np.float32)
    b = rng.random(parent_b, dtype=np.float32)
    oracle.copy(counter, a.reshape(-1), parent_a, b.reshape(-1), parent_b,
                dst_base=int(np.ravel_multi_index(sa, parent_a)),
                src_base=int(np.ravel_multi_index(sb, parent_b)))
    want = np.zeros(parent_a, dtype=np.float32)
    want[_sl(counter, sa)] = b[_sl(counter, sb)]
    assert want.tobytes() == a.tobytes()


def test_embed_invariants_mass_crop_special_values():
    rng = np.random.default_rng(11)
    src_s, dst_s = (5, 6, 7), (8, 9, 11)
    src = rng.random(src_s, dtype=np.float32)
    src.reshape(-1)[:8] = np.array([0.0, -0.0, np.inf, -np.inf, 1e-45, -1e-40, 3.0, 0.0],
                                   dtype=np.float32)
    # A NaN with a payload: the copy moves bits, so the payload survives.
    src.reshape(-1)[8:9].view(np.uint32)[0] = 0x7FC01234
    dst = np.zeros(dst_s, dtype=np.float32)
    oracle.copy(src_s, dst.reshape(-1), dst_s, src.reshape(-1), src_s)
    # mass: same non-zeros and bit-identical sequential float64 sums
    # (the origin embedding keeps the row-major order of the non-zeros).
    assert np.count_nonzero(dst) == np.count_nonzero(src)
    fin_s = src.reshape(-1)[np.isfinite(src.reshape(-1))].astype(np.float64)
    fin_d = dst.reshape(-1)[np.isfinite(dst.reshape(-1))].astype(np.float64)
    assert float(np.add.reduce(fin_d[fin_d != 0])) == float(np.add.reduce(fin_s[fin_s != 0]))
    # crop(embed(x)) == x bit for bit
    back = np.zeros(src_s, dtype=np.float32)
    oracle.copy(src_s, back.reshape(-1), src_s, dst.reshape(-1), dst_s)
    assert back.tobytes() == src.tobytes()


def test_copy_float64_elements():
    rng = np.random.default_rng(5)
    y = rng.standard_normal((6, 5, 4))
    x = np.zeros((4, 5, 2))
    oracle.copy((4, 5, 2), x.reshape(-1), (4, 5, 2), y.reshape(-1), (6, 5, 4))
    assert np.array(y[:4, :5, :2]).tobytes() == x.tobytes()


@pytest.mark.parametrize("seed", range(5))
def test_embed_fill_matches_np_pad(seed):
    rng = np.random.default_rng(200 + seed)
    d = int(rng.integers(1, 5))
    src_s, dst_s = _rand_shapes(rng, d, pad_hi=6)
    src = rng.standard_normal(src_s).astype(np.float32)
    dst = np.full(dst_s, 7.0, dtype=np.float32)      # garbage to be overwritten
    oracle.embed_fill(dst_s, dst.reshape(-1), dst_s, src.reshape(-1), src_s)
    want = np.pad(src, [(0, b - a) for a, b in zip(src_s, dst_s)])
    assert want.tobytes() == dst.tobytes()
    # == zero fill followed by a copy over the source shape
    z = np.zeros(dst_s, dtype=np.float32)
    oracle.copy(src_s, z.reshape(-1), dst_s, src.reshape(-1), src_s)
    assert z.tobytes() == dst.tobytes()


def _three(rng, d):
    x_s = tuple(int(v) for v in rng.integers(1, 7, size=d))
    y_s = tuple(s + int(rng.integers(0, 4)) for s in x_s)
    z_s = tuple(s + int(rng.integers(0, 4)) for s in x_s)
    return x_s, y_s, z_s


@pytest.mark.parametrize("seed", range(8))
def test_mul_acc_matches_numpy_float32(seed):
    rng = np.random.default_rng(300 + seed)
    d = int(rng.integers(1, 6))
    x_s, y_s, z_s = _three(rng, d)
    x = rng.random(x_s, dtype=np.float32)
    y = rng.standard_normal(y_s).astype(np.float32)
    z = rng.standard_normal(z_s).astype(np.float32)
    want = x.copy()
    want += y[_sl(x_s)] * z[_sl(x_s)]           # numpy: product, then sum
    oracle.mul_acc(x_s, x.reshape(-1), x_s, y.reshape(-1), y_s, z.reshape(-1), z_s)
    assert want.tobytes() == x.tobytes()


def test_mul_acc_two_roundings_not_fma():
    # y = z = 1 + 2^-12: the exact product 1 + 2^-11 + 2^-24 is a tie in
    # float32 and rounds to the even neighbour 1 + 2^-11, so
    # -(1 + 2^-11) + fl(y*z) is exactly 0; a fused multiply-add would
    # leave 2^-24 instead.
    e = np.float32(2.0 ** -12)
    x = np.array([-(1 + 2 * e)], dtype=np.float32)
    y = np.array([1 + e], dtype=np.float32)
    z = np.array([1 + e], dtype=np.float32)
    oracle.mul_acc((1,), x, (1,), y, (1,), z, (1,))
    assert x[0] == 0.0


def test_mul_acc_special_cases_and_untouched_points():
    rng = np.random.default_rng(9)
    x_s, big = (4, 5, 6), (6, 7, 8)
    x = rng.random(big, dtype=np.float32)
    x0 = x.copy()
    y = np.zeros(big, dtype=np.float32)
    z = rng.random(big, dtype=np.float32)
    # y = 0: x unchanged bit for bit (x is positive, so x + 0 == x).
    oracle.mul_acc(x_s, x.reshape(-1), big, y.reshape(-1), big, z.reshape(-1), big)
    assert x.tobytes() == x0.tobytes()
    # z = 1: x + y over the counter, and nothing outside the counter moves.
    y = rng.random(big, dtype=np.float32)
    one = np.ones(big, dtype=np.float32)
    oracle.mul_acc(x_s, x.reshape(-1), big, y.reshape(-1), big, one.reshape(-1), big)
    want = x0.copy()
    want[_sl(x_s)] = x0[_sl(x_s)] + y[_sl(x_s)]
    assert want.tobytes() == x.tobytes()


def test_mul_acc_aliased_update():
    # x[t] += y[t] * x[t] with x passed twice (legal: Section 4, aliasing).
    rng = np.random.default_rng(4)
    x = rng.random((5, 6), dtype=np.float32)
    y = rng.random((7, 8), dtype=np.float32)
    want = x.copy()
    want += y[:5, :6] * x
    oracle.mul_acc((5, 6), x.reshape(-1), (5, 6), y.reshape(-1), (7, 8), x.reshape(-1), (5, 6))
    assert want.tobytes() == x.tobytes()


@pytest.mark.parametrize("f64", [False, True])
def test_mul_matches_numpy(f64):
    rng = np.random.default_rng(12)
    dt = np.float64 if f64 else np.float32
    i_s, a_s, b_s = (3, 4, 5), (5, 4, 7), (3, 6, 5)
    a = rng.standard_normal(a_s).astype(dt)
    b = rng.standard_normal(b_s).astype(dt)
    out = np.zeros(i_s, dtype=dt)
    oracle.mul(i_s, out.reshape(-1), i_s, a.reshape(-1), a_s, b.reshape(-1), b_s)
    assert (a[_sl(i_s)] * b[_sl(i_s)]).tobytes() == out.tobytes()


def test_mul_adj_matches_numpy():
    rng = np.random.default_rng(13)
    sa, sb, si = (6, 5, 7), (4, 6, 7), (4, 5, 6)
    a = rng.standard_normal(sa).astype(np.float32)
    b = rng.standard_normal(sb).astype(np.float32)
    g = rng.standard_normal(si).astype(np.float32)
    ga = np.full(sa, 9.0, dtype=np.float32)
    gb = np.full(sb, 9.0, dtype=np.float32)
    oracle.mul_adj(ga.reshape(-1), sa, gb.reshape(-1), sb, g.reshape(-1), si,
                   a.reshape(-1), b.reshape(-1))
    wa = np.zeros(sa, dtype=np.float32)
    wa[_sl(si)] = g * b[_sl(si)]
    wb = np.zeros(sb, dtype=np.float32)
    wb[_sl(si)] = g * a[_sl(si)]
    assert wa.tobytes() == ga.tobytes()
    assert wb.tobytes() == gb.tobytes()


def test_bounds_are_checked_once_per_call():
    a = np.zeros((4, 4), dtype=np.float32)
    b = np.zeros((3, 5), dtype=np.float32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.copy((4, 4), a.reshape(-1), (4, 4), b.reshape(-1), (3, 5))
    assert e.value.code == oracle.EBOUNDS
    with pytest.raises(oracle.OracleError):
        oracle.mul_acc((4, 5), a.reshape(-1), (4, 4), a.reshape(-1), (4, 4), a.reshape(-1), (4, 4))


def test_zero_extent_is_a_no_op():
    a = np.full((4, 4), 3.0, dtype=np.float32)
    b = np.zeros((4, 4), dtype=np.float32)
    oracle.copy((4, 0), a.reshape(-1), (4, 4), b.reshape(-1), (4, 4))
    assert (a == 3.0).all()
