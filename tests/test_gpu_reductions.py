"""GPU parity for benchmarks 2-4 of Section 3 and the tuple-reading
reductions of Section 2, against the CPU oracle on the same seeded inputs:

- benchmark 3's update x <- x + y*x - z and the nonzero bounding box are
  bit-exact;
- the naive convolution is bit-exact (the GPU adds every output's terms in
  the paper's loop order);
- the inner product and marginals are float64 sums in another order: they
  must lie within the sequential-summation bound n*eps*sum|w| of the
  oracle's value (exact for integer-valued inputs), and the float32 result
  within one float32 rounding of it."""
import numpy as np
import pytest
import torch

import oracle
from paper_1608_00099_amd import _lib as L
from paper_1608_00099_amd import api, inputs
from tests.gpu_util import announce, bits_equal, dev, first_mismatch, host

pytestmark = pytest.mark.gpu

EPS64 = np.finfo(np.float64).eps


def _close64(got, want, n, mag):
    return abs(float(got) - float(want)) <= max(n, 1) * EPS64 * float(mag) + 1e-300


def _close32(got32, want64, n, mag):
    # within one float32 rounding of a value inside the float64 bound
    slack = max(n, 1) * EPS64 * float(mag)
    ulp = np.spacing(np.float32(abs(want64) + slack))
    return abs(float(got32) - float(want64)) <= float(ulp) + slack


# ---------------------------------------------------------------------------
# Inner product (benchmark 2)
# ---------------------------------------------------------------------------

DOT_CASES = [
    ((37, 41), (40, 39)),
    ((9, 8, 7, 6), (10, 7, 9, 5)),
    ((64, 48), (64, 48)),
    ((3, 1, 300), (2, 5, 301)),
    ((1 << 16,), (70000,)),
]


@pytest.mark.parametrize("case", range(len(DOT_CASES)))
def test_dot_matches_oracle(case):
    sa, sb = DOT_CASES[case]
    announce("dot", sa, sb)
    rng = np.random.default_rng(200 + case)
    a = rng.standard_normal(sa).astype(np.float32)
    b = rng.standard_normal(sb).astype(np.float32)
    counter = tuple(min(x, y) for x, y in zip(sa, sb))
    want = oracle.dot(counter, [a, b], [sa, sb])
    mag = oracle.dot(counter, [np.abs(a), np.abs(b)], [sa, sb])
    n = int(np.prod(counter))
    o32, o64 = api.dot(dev(a), dev(b))
    assert _close64(host(o64)[0], want, n, mag), (host(o64)[0], want)
    assert _close32(host(o32)[0], want, n, mag)


def test_dot_integer_values_exact_and_three_operands():
    announce("dot exact")
    rng = np.random.default_rng(210)
    a = rng.integers(-3, 4, size=(33, 17, 9)).astype(np.float32)
    b = rng.integers(-3, 4, size=(30, 20, 9)).astype(np.float32)
    c = rng.integers(-3, 4, size=(31, 17, 12)).astype(np.float32)
    counter = (30, 17, 9)
    want = oracle.dot(counter, [a, b, c], [a.shape, b.shape, c.shape])
    o32, o64 = api.dot(dev(a), dev(b), dev(c))
    assert host(o64)[0] == want and host(o32)[0] == np.float32(want)


def test_dot_benchmark2_full_size():
    # (2^10, 2^9, 2^8) . (2^9, 2^9, 2^5) over the 2^23 shared tuples
    sa, sb = (1 << 10, 1 << 9, 1 << 8), (1 << 9, 1 << 9, 1 << 5)
    announce("dot benchmark 2", sa, sb)
    a = inputs.uniform(7, sa, 1)
    b = inputs.uniform(7, sb, 2)
    counter = (1 << 9, 1 << 9, 1 << 5)
    want = oracle.dot(counter, [a, b], [sa, sb])
    o32, o64 = api.dot(dev(a), dev(b))
    n = 1 << 23
    assert _close64(host(o64)[0], want, n, want)          # positive terms: sum|w| = want
    assert _close32(host(o32)[0], want, n, want)


def test_dot_degenerate():
    announce("dot degenerate")
    a = torch.full((), 2.5, device="cuda")
    b = torch.full((), -4.0, device="cuda")
    o32, o64 = api.dot(a, b)
    assert host(o64)[0] == -10.0
    z = torch.ones((3, 0), device="cuda")
    st = L.triot_apply(L.OP_DOT, 2, 2, [(3, 0), (3, 0)], None, [z.data_ptr(), z.data_ptr()],
                       None, None, 0, 0, 0, 0)
    assert st == L.OK


# ---------------------------------------------------------------------------
# Benchmark 3's update
# ---------------------------------------------------------------------------

def test_xpyx_mz_benchmark3_shapes_bit_exact():
    xs, ys, zs = (129, 32, 13, 16), (253, 64, 64, 23), (256, 39, 64, 33)
    announce("xpyx_mz benchmark 3", xs, ys, zs)
    rng = np.random.default_rng(220)
    x = rng.standard_normal(xs).astype(np.float32)
    y = rng.standard_normal(ys).astype(np.float32)
    z = rng.standard_normal(zs).astype(np.float32)
    want = x.copy()
    oracle.xpyx_mz(xs, want, xs, y, ys, z, zs)
    gx = dev(x)
    api.xpyx_mz_(gx, dev(y), dev(z))
    got = host(gx)
    assert bits_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("d", [2, 4, 6, 8])
def test_xpyx_mz_sweep_and_special_values(d):
    xs, ys, zs = inputs.cfg2_inter_shapes(d, log2_target=15)
    announce("xpyx_mz sweep", d, xs, ys, zs)
    rng = np.random.default_rng(230 + d)
    x = rng.standard_normal(xs).astype(np.float32)
    y = rng.standard_normal(ys).astype(np.float32)
    z = rng.standard_normal(zs).astype(np.float32)
    xf = x.reshape(-1)
    xf[:5] = [np.inf, -0.0, 1e-45, np.nan, -3e-39]
    want = x.copy()
    oracle.xpyx_mz(xs, want, xs, y, ys, z, zs)
    gx = dev(x)
    api.xpyx_mz_(gx, dev(y), dev(z))
    got = host(gx)
    assert bits_equal(got, want), first_mismatch(got, want)


def test_xpyx_mz_not_fused_and_windows():
    announce("xpyx_mz fused check")
    e = np.float32(2.0 ** -12)
    x = np.array([1 + e] * 8, np.float32)
    y = np.array([-(1 + e)] * 8, np.float32)
    z = np.zeros(8, np.float32)
    gx = dev(x)
    api.xpyx_mz_(gx, dev(y), dev(z))
    assert np.all(host(gx) == np.float32(-(2.0 ** -12)))
    rng = np.random.default_rng(240)
    px, py, pz = (10, 9, 12), (12, 14, 13), (9, 20, 15)
    c = (4, 6, 7)
    bx, by, bz = 2 * 108 + 3 * 12 + 1, 5 * 182 + 7 * 13 + 2, 1 * 300 + 11 * 15 + 3
    X = rng.standard_normal(px).astype(np.float32)
    Y = rng.standard_normal(py).astype(np.float32)
    Z = rng.standard_normal(pz).astype(np.float32)
    want = X.copy()
    oracle.xpyx_mz(c, want, px, Y, py, Z, pz, bx, by, bz)
    gx = dev(X)
    api.xpyx_mz_(gx, dev(Y), dev(Z), counter=c, shapes=[px, py, pz], bases=[bx, by, bz])
    got = host(gx)
    assert bits_equal(got, want), first_mismatch(got, want)


# ---------------------------------------------------------------------------
# Marginalization
# ---------------------------------------------------------------------------

MARG_CASES = [
    # (shapes, keep)
    ([(16, 16, 16, 16, 16, 16)], (1, 0, 0, 0, 0, 0)),     # one axis kept: 16 outputs, many parts
    ([(16, 16, 16, 16, 16, 16)], (0, 0, 1, 0, 1, 0)),
    ([(16, 16, 16, 16, 16, 16)], (1, 1, 1, 1, 1, 0)),     # innermost reduced
    ([(40, 30, 20)], (0, 1, 1)),
    ([(7, 300, 5)], (1, 0, 1)),
    ([(9, 8, 7, 6), (10, 7, 9, 5)], (1, 0, 1, 0)),        # two operands over the intersection
    ([(5, 1, 6, 1, 7)], (1, 1, 0, 0, 1)),                  # extent-1 axes kept and reduced
    ([(33, 35)], (0, 0)),                                   # nothing kept
    ([(33, 35)], (1, 1)),                                   # everything kept
]


@pytest.mark.parametrize("case", range(len(MARG_CASES)))
def test_marginal_matches_oracle(case):
    shapes, keep = MARG_CASES[case]
    announce("marginal", shapes, keep)
    rng = np.random.default_rng(250 + case)
    ts = [rng.random(s).astype(np.float32) for s in shapes]
    counter = tuple(min(s[i] for s in shapes) for i in range(len(shapes[0])))
    want = oracle.marginal(counter, keep, ts, shapes)
    g = [dev(t) for t in ts]
    o32, o64 = api.marginal(g[0], keep, others=g[1:])
    got64, got32 = host(o64), host(o32)
    assert got64.shape == want.shape
    nred = int(np.prod([c for c, k in zip(counter, keep) if not k] or [1]))
    # positive weights: sum|w| is the value itself
    bound = nred * EPS64 * np.abs(want)
    assert np.all(np.abs(got64 - want) <= bound + 1e-300)
    ulp = np.spacing(np.abs(want + bound).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(got32.astype(np.float64) - want) <= ulp + bound)


# One contiguous reduced run per kept tuple, walked interleaved (lane l of a
# chunk takes every 64th element): ragged last chunks, one and two
# operands; integer values make every order of summation exact.
@pytest.mark.parametrize("shape,keep", [((3, 1028), (1, 0)), ((5, 4100), (1, 0)),
                                        ((2, 3, 16, 64), (1, 1, 0, 0)), ((3, 2051), (1, 0)),
                                        ((1, 70000), (1, 0)), ((6, 8, 1, 2048), (1, 0, 0, 0))])
def test_marginal_interleaved_runs(shape, keep):
    announce("marginal interleaved", shape, keep)
    rng = inputs.rng(3, 23, len(shape), int(np.prod(shape)))
    a = rng.integers(0, 5, size=shape).astype(np.float32)
    b = rng.integers(-2, 3, size=shape).astype(np.float32)
    for ts in ([a], [a, b]):
        want = oracle.marginal(shape, keep, ts, [shape] * len(ts))
        o32, o64 = api.marginal(dev(ts[0]), keep, others=[dev(t) for t in ts[1:]])
        assert np.array_equal(host(o64), want), (shape, keep, len(ts))
        assert np.array_equal(host(o32), want.astype(np.float32))


# A kept innermost axis (the column walk: four outputs per lane, rows
# interleaved over the parts) and its near misses: output counts not a
# multiple of 4, a kept axis that is not unit-stride in every operand,
# two operands, rows not a multiple of the parts.
@pytest.mark.parametrize("shapes,keep", [
    ([(16, 16, 16, 16, 16, 16)], (0, 0, 0, 0, 0, 1)),
    ([(300, 64)], (0, 1)),
    ([(7, 40, 12)], (0, 0, 1)),
    ([(7, 40, 12), (7, 40, 12)], (0, 0, 1)),
    ([(1001, 8)], (0, 1)),
    ([(513, 10)], (0, 1)),
    ([(40, 30, 20), (41, 30, 22)], (0, 0, 1)),
])
def test_marginal_kept_inner(shapes, keep):
    announce("marginal kept inner", shapes, keep)
    rng = inputs.rng(3, 26, len(shapes), len(shapes[0]), int(np.prod(shapes[0])))
    ts = [rng.integers(0, 5, size=s).astype(np.float32) for s in shapes]
    counter = tuple(min(s[i] for s in shapes) for i in range(len(shapes[0])))
    want = oracle.marginal(counter, keep, ts, shapes)
    o32, o64 = api.marginal(dev(ts[0]), keep, others=[dev(t) for t in ts[1:]])
    assert np.array_equal(host(o64), want)
    assert np.array_equal(host(o32), want.astype(np.float32))
    # real values: within the summation bound
    tr = [rng.random(s).astype(np.float32) for s in shapes]
    want = oracle.marginal(counter, keep, tr, shapes)
    o32, o64 = api.marginal(dev(tr[0]), keep, others=[dev(t) for t in tr[1:]])
    nred = int(np.prod([c for c, k in zip(counter, keep) if not k] or [1]))
    assert np.all(np.abs(host(o64) - want) <= nred * EPS64 * np.abs(want) + 1e-300)


# Short reduced runs (innermost, unit-stride, 4 .. 64 elements: a lane group
# per output, one word quad per lane, butterflies): every run length, a
# window of a wider operand, two operands, an output count that leaves the
# last wave part empty.
@pytest.mark.parametrize("shapes,keep", [
    ([(70000, 4)], (1, 0)),
    ([(40000, 8), (40000, 8)], (1, 0)),
    ([(17000, 16)], (1, 0)),
    ([(8193, 32)], (1, 0)),
    ([(4099, 64)], (1, 0)),
    ([(4100, 20), (4100, 16)], (1, 0)),
    ([(5, 7, 1000, 16)], (1, 1, 1, 0)),
])
def test_marginal_short_runs(shapes, keep):
    announce("marginal short runs", shapes, keep)
    rng = inputs.rng(3, 27, len(shapes), int(np.prod(shapes[0])))
    ts = [rng.integers(0, 5, size=s).astype(np.float32) for s in shapes]
    counter = tuple(min(s[i] for s in shapes) for i in range(len(shapes[0])))
    want = oracle.marginal(counter, keep, ts, shapes)
    o32, o64 = api.marginal(dev(ts[0]), keep, others=[dev(t) for t in ts[1:]])
    assert np.array_equal(host(o64), want)
    assert np.array_equal(host(o32), want.astype(np.float32))
    tr = [rng.random(s).astype(np.float32) for s in shapes]
    want = oracle.marginal(counter, keep, tr, shapes)
    o32, o64 = api.marginal(dev(tr[0]), keep, others=[dev(t) for t in tr[1:]])
    nred = int(np.prod([c for c, k in zip(counter, keep) if not k] or [1]))
    assert np.all(np.abs(host(o64) - want) <= nred * EPS64 * np.abs(want) + 1e-300)


def test_marginal_integer_values_exact():
    announce("marginal exact")
    rng = np.random.default_rng(270)
    a = rng.integers(0, 5, size=(20, 30, 40)).astype(np.float32)
    b = rng.integers(0, 5, size=(22, 30, 41)).astype(np.float32)
    for keep in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (0, 0, 0)]:
        want = oracle.marginal((20, 30, 40), keep, [a, b], [a.shape, b.shape])
        o32, o64 = api.marginal(dev(a), keep, others=[dev(b)])
        assert np.array_equal(host(o64), want), keep
        assert np.array_equal(host(o32), want.astype(np.float32)), keep


# ---------------------------------------------------------------------------
# Nonzero bounding box
# ---------------------------------------------------------------------------

BBOX_CASES = [
    [(40, 50, 60)],
    [(16, 16, 16, 16, 16, 16)],
    [(9, 8, 7, 6), (10, 7, 9, 5)],
    [(3, 1, 300), (2, 5, 301)],
    [(5000,)],
    [(2, 3, 2, 3, 2, 3, 2, 3, 2, 3)],
]


@pytest.mark.parametrize("case", range(len(BBOX_CASES)))
@pytest.mark.parametrize("density", [0.0, 1e-4, 0.05])
def test_bbox_matches_oracle(case, density):
    shapes = BBOX_CASES[case]
    announce("bbox", shapes, density)
    rng = np.random.default_rng(280 + case)
    ts = []
    for s in shapes:
        v = rng.standard_normal(s).astype(np.float32)
        v[rng.random(s) >= max(density, 0.5 if len(ts) else density)] = 0.0
        ts.append(v)
    counter = tuple(min(s[i] for s in shapes) for i in range(len(shapes[0])))
    want = oracle.bbox(counter, ts, shapes)
    got = host(api.bbox(*[dev(t) for t in ts]))
    assert np.array_equal(got, want), (got, want)


# Rows of 4, 8 or 16 words laid end to end (staged tile loads; rows of 16
# words as quads of 16 rows per load, masks combined across lanes): one to
# three operands, sparse and denser, and single nonzeros at the first and
# last point (a ragged last wave: 1, 15, 17 or 63 of its 64 rows).
@pytest.mark.parametrize("shape", [(7, 5, 16), (33, 29, 16), (300, 8), (5, 77, 4),
                                   (2, 3, 1, 4, 3, 8), (65, 8, 16), (1, 16), (17, 16),
                                   (1041, 16), (2, 3, 5, 7, 16)])
@pytest.mark.parametrize("density", [1e-3, 0.05])
def test_bbox_short_rows(shape, density):
    announce("bbox short rows", shape, density)
    rng = inputs.rng(3, 22, len(shape), int(np.prod(shape)), int(density * 1e4))
    a = rng.standard_normal(shape).astype(np.float32)
    b = rng.standard_normal(shape).astype(np.float32)
    a[rng.random(shape) >= density] = 0.0
    b[rng.random(shape) >= 0.5] = 0.0
    c3 = rng.standard_normal(shape).astype(np.float32)
    c3[rng.random(shape) >= 0.9] = 0.0
    for ts in ([a], [a, b], [a, b, c3]):
        want = oracle.bbox(shape, ts, [shape] * len(ts))
        got = host(api.bbox(*[dev(t) for t in ts]))
        assert np.array_equal(got, want), (ts is None, got, want)
    for corner in (0, -1):
        c = np.zeros(shape, np.float32)
        c.reshape(-1)[corner] = 3.0
        want = oracle.bbox(shape, [c], [shape])
        got = host(api.bbox(dev(c)))
        assert np.array_equal(got, want), (corner, got, want)


# Rows a multiple of 32 words laid end to end: both halves of every 32-word
# segment through one staged pass; one and two operands, single nonzeros at
# the first and last point and inside the second half of a segment.
@pytest.mark.parametrize("shape", [(5, 32), (33, 7, 64), (256, 256), (3, 5, 7, 96)])
def test_bbox_32_word_segments(shape):
    announce("bbox 32-word segments", shape)
    rng = inputs.rng(3, 29, len(shape), int(np.prod(shape)))
    a = rng.standard_normal(shape).astype(np.float32)
    b = rng.standard_normal(shape).astype(np.float32)
    a[rng.random(shape) >= 0.01] = 0.0
    b[rng.random(shape) >= 0.5] = 0.0
    for ts in ([a], [a, b]):
        want = oracle.bbox(shape, ts, [shape] * len(ts))
        got = host(api.bbox(*[dev(t) for t in ts]))
        assert np.array_equal(got, want), (got, want)
    n = int(np.prod(shape))
    for idx in (0, n - 1, 21, n - 7):
        c = np.zeros(shape, np.float32)
        c.reshape(-1)[idx] = -2.0
        want = oracle.bbox(shape, [c], [shape])
        got = host(api.bbox(dev(c)))
        assert np.array_equal(got, want), (idx, got, want)


def test_bbox_special_values_and_underflowing_products():
    announce("bbox special")
    a = np.zeros((6, 70), np.float32)
    b = np.zeros((6, 70), np.float32)
    a[1, 3], b[1, 3] = 1e-30, 1e-30        # the float32 product underflows; still nonzero
    a[4, 60], b[4, 60] = np.nan, 2.0        # NaN counts as nonzero
    a[5, 65], b[5, 65] = -0.0, 1.0          # -0.0 is zero
    want = oracle.bbox((6, 70), [a, b], [a.shape, b.shape])
    assert np.array_equal(want, [[1, 4], [3, 60]])
    got = host(api.bbox(dev(a), dev(b)))
    assert np.array_equal(got, want)


# ---------------------------------------------------------------------------
# Naive convolution (benchmark 4)
# ---------------------------------------------------------------------------

CONV_CASES = [
    ((256, 8), (256, 8)),               # benchmark 4
    ((37,), (5,)),
    ((4, 6, 5), (3, 2, 7)),
    ((1, 9, 1), (3, 1, 4)),
    ((100, 100), (5, 5)),               # inputs beyond the LDS staging size
    ((2, 3, 2, 3), (3, 2, 3, 2)),
    ((), ()),
]


@pytest.mark.parametrize("case", range(len(CONV_CASES)))
def test_conv_bit_exact(case):
    ls, rs = CONV_CASES[case]
    announce("conv", ls, rs)
    rng = np.random.default_rng(300 + case)
    l = np.ascontiguousarray(rng.standard_normal(ls))
    r = np.ascontiguousarray(rng.standard_normal(rs))
    want = oracle.conv(l, r)
    got = host(api.conv(dev(l), dev(r)))
    assert bits_equal(got, want), first_mismatch(got, want)


# Signed zeros, subnormal products and overflow to +inf, bit for bit (no
# invalid operation, so no NaN whose payload could differ between the host
# and the GPU).
@pytest.mark.parametrize("ls,rs", [((256, 8), (256, 8)), ((37,), (5,)), ((4, 6, 5), (3, 2, 7)),
                                   ((100, 100), (5, 5))])
def test_conv_signed_zeros_subnormals_overflow(ls, rs):
    announce("conv special", ls, rs)
    rng = np.random.default_rng(320 + len(ls))
    l = rng.standard_normal(ls)
    r = rng.standard_normal(rs)
    lf, rf = l.reshape(-1), r.reshape(-1)
    pick = rng.random(lf.size)
    lf[pick < 0.3] = 0.0
    lf[(pick >= 0.3) & (pick < 0.5)] = -0.0
    lf[(pick >= 0.5) & (pick < 0.55)] = 1e-300
    rf[rng.random(rf.size) < 0.2] = -0.0
    rf[rng.random(rf.size) < 0.05] = 1e-20          # subnormal products with 1e-300
    want = oracle.conv(np.ascontiguousarray(l), np.ascontiguousarray(r))
    got = host(api.conv(dev(l), dev(r)))
    assert bits_equal(got, want), first_mismatch(got, want)
    # overflow: all-positive huge values sum to +inf
    big_l = np.full(ls, 1e306)
    big_r = np.abs(r) + 1.0
    want = oracle.conv(big_l, np.ascontiguousarray(big_r))
    got = host(api.conv(dev(big_l), dev(big_r)))
    assert bits_equal(got, want), first_mismatch(got, want)


def test_conv_rejects_bad_shapes_and_aliasing():
    announce("conv errors")
    l = torch.zeros((4, 5), dtype=torch.float64, device="cuda")
    r = torch.zeros((3, 2), dtype=torch.float64, device="cuda")
    out = torch.zeros((6, 6), dtype=torch.float64, device="cuda")   # should be (6, 6): ok
    api.conv(l, r, out=out)
    bad = torch.zeros((6, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(L.TriotError) as e:
        api.apply(L.OP_CONV, [bad, l, r], [(6, 5), (4, 5), (3, 2)], None, None, None)
    assert e.value.status == L.E_BOUNDS
    big = torch.zeros(100, dtype=torch.float64, device="cuda")
    with pytest.raises(L.TriotError) as e:
        api.apply(L.OP_CONV, [big, big, r], [(6, 6), (4, 5), (3, 2)], None, None, None)
    assert e.value.status == L.E_ALIAS
