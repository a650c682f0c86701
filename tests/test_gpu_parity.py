"""GPU kernels against the CPU oracle, element by element, on the same seeded
inputs: bit-exact for copies, index arithmetic and the float32 element-wise
ops; moments within 1e-6 relative of the float64 oracle.

Sizes are chosen so the oracle finishes in seconds while the kernels still
run several work units with ragged tails; the full benchmark sizes are
covered by tests/test_gpu_fullsize.py."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1608_00099_amd import _lib as L
from paper_1608_00099_amd import api, inputs
from tests.gpu_util import announce, bits_equal, dev, first_mismatch, host, rel_err

pytestmark = pytest.mark.gpu


def _prod(s):
    return int(np.prod(s, dtype=np.int64)) if len(s) else 1


# ---------------------------------------------------------------------------
# Index arithmetic
# ---------------------------------------------------------------------------

INDEX_CASES = [
    # (counter, shapes, bases)
    ((4, 9, 7, 5), [(4, 9, 7, 5), (5, 10, 8, 6)], None),          # the worked example's shape
    ((48, 40, 36), [(64, 64, 64), (48, 40, 36)], None),
    ((3, 1, 5, 1, 7), [(4, 2, 6, 3, 9), (3, 1, 5, 1, 7), (5, 1, 8, 2, 7)], None),
    ((6, 5, 4, 3, 2, 3, 2, 2), [(7, 6, 5, 4, 3, 4, 3, 3)] * 2, None),
    ((2,) * 12, [(3,) * 12, (2,) * 12], None),
    ((5, 6, 7), [(9, 9, 9), (8, 7, 10)], [2 * 81 + 1 * 9 + 2, 1 * 70 + 0 + 3]),
    ((1 << 20,), [(1 << 20,), (3 << 20,)], [0, 12345]),
    ((3, 70000), [(4, 70001), (3, 70000)], None),
    ((), [(), ()], [0, 0]),
    ((7,), [(7,)], None),
]


@pytest.mark.parametrize("case", range(len(INDEX_CASES)))
def test_index_bit_exact(case):
    counter, shapes, bases = INDEX_CASES[case]
    announce("index", counter, shapes, bases)
    got = host(api.index(shapes, counter, bases))
    want = oracle.index(counter, shapes, bases)
    assert got.shape == want.shape
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_index_worked_example_651():
    announce("index 651")
    got = host(api.index([(4, 9, 7, 5)], (4, 9, 7, 5)))
    f = oracle.unflatten(651, (4, 9, 7, 5))
    assert f == (2, 0, 4, 1)
    assert got[0, 651] == 651
    # the same tuple in a larger operand, as the GPU co-iterates both
    got = host(api.index([(4, 9, 7, 5), (8, 16, 8, 8)], (4, 9, 7, 5)))
    assert got[1, 651] == 2081


@pytest.mark.parametrize("d", range(1, 9))
def test_index_runtime_dimension_sweep(d):
    src, dst = inputs.cfg2_pad_shapes(d, log2_target=14)
    announce("index sweep", d, src, dst)
    got = host(api.index([dst, src], src))
    want = oracle.index(src, [dst, src])
    assert np.array_equal(got, want), first_mismatch(got, want)


# ---------------------------------------------------------------------------
# Copies
# ---------------------------------------------------------------------------

def test_copy_cfg1_pad_embed_bit_exact():
    announce("copy cfg1")
    src = inputs.cfg1_values()
    dst = np.zeros(inputs.CFG1_DST, dtype=np.float32)
    want = dst.copy()
    oracle.copy(inputs.CFG1_SRC, want.reshape(-1), inputs.CFG1_DST, src.reshape(-1), inputs.CFG1_SRC)
    g = dev(dst)
    api.pad_embed_into(g, dev(src))
    got = host(g)
    assert bits_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("d", range(2, 9))
@pytest.mark.parametrize("log2n", [12, 17])
def test_copy_pad_embed_sweep(d, log2n):
    src_s, dst_s = inputs.cfg2_pad_shapes(d, log2_target=log2n)
    announce("copy sweep", d, src_s, dst_s)
    src = inputs.uniform(2, src_s, 10, d, log2n)
    want = np.zeros(dst_s, dtype=np.float32)
    oracle.copy(src_s, want.reshape(-1), dst_s, src.reshape(-1), src_s)
    g = torch.zeros(dst_s, dtype=torch.float32, device="cuda")
    api.pad_embed_into(g, dev(src))
    got = host(g)
    assert bits_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("d", [2, 3, 5])
def test_copy_crop_float64(d):
    src_s, dst_s = inputs.cfg2_pad_shapes(d, log2_target=14)
    announce("crop f64", d)
    big = inputs.rng(2, 20, d).standard_normal(dst_s)
    want = np.full(src_s, np.nan)
    oracle.copy(src_s, want.reshape(-1), src_s, big.reshape(-1), dst_s)
    got = host(api.crop(dev(big), src_s))
    assert bits_equal(got, want), first_mismatch(got, want)


def test_copy_windows_with_bases_and_special_values():
    announce("copy windows")
    rng = np.random.default_rng(5)
    pa, pb, counter = (9, 10, 11, 12), (8, 13, 9, 14), (4, 6, 5, 7)
    sa, sb = (3, 2, 4, 1), (2, 5, 1, 6)
    ba, bb = int(np.ravel_multi_index(sa, pa)), int(np.ravel_multi_index(sb, pb))
    a = np.zeros(pa, dtype=np.float32)
    b = rng.standard_normal(pb).astype(np.float32)
    bf = b.reshape(-1)
    bf[:6] = np.array([np.nan, -0.0, np.inf, -np.inf, 1e-45, -3e-39], dtype=np.float32)
    bf[6:7].view(np.uint32)[0] = 0x7FA00001       # signalling-NaN payload
    b[sb[0], sb[1], sb[2], sb[3]] = np.float32(1e-44)
    want = a.copy()
    oracle.copy(counter, want.reshape(-1), pa, b.reshape(-1), pb, ba, bb)
    g = dev(a)
    api.copy_(g, dev(b), counter=counter, dst_base=ba, src_base=bb)
    got = host(g)
    assert bits_equal(got, want), first_mismatch(got, want)


def test_copy_vector_widths():
    # aligned shapes use 16- and 8-byte lanes; results must not change
    for src_s, dst_s in [((64, 48), (64, 64)), ((10, 6), (12, 10)), ((7, 33, 4), (9, 40, 8)),
                         ((3, 5), (4, 7))]:
        announce("copy vec", src_s, dst_s)
        src = inputs.uniform(2, src_s, 30)
        want = np.zeros(dst_s, dtype=np.float32)
        oracle.copy(src_s, want.reshape(-1), dst_s, src.reshape(-1), src_s)
        g = torch.zeros(dst_s, dtype=torch.float32, device="cuda")
        api.pad_embed_into(g, dev(src))
        got = host(g)
        assert bits_equal(got, want), (src_s, first_mismatch(got, want))


def test_copy_degenerate():
    announce("copy degenerate")
    # scalar (d = 0)
    a = torch.zeros((), device="cuda")
    b = torch.full((), 3.5, device="cuda")
    api.copy_(a, b)
    assert host(a) == 3.5
    # extent 0: nothing happens
    a = torch.full((4, 4), 7.0, device="cuda")
    api.copy_(a, torch.zeros((4, 4), device="cuda"), counter=(4, 0))
    assert (host(a) == 7.0).all()
    # all extent-1 axes
    a = torch.zeros((1, 1, 1), device="cuda")
    api.copy_(a, torch.full((1, 1, 1), 2.0, device="cuda"))
    assert host(a).reshape(-1)[0] == 2.0


def test_copy_aliasing_rejected():
    announce("copy alias")
    x = torch.zeros(64, device="cuda")
    with pytest.raises(L.TriotError) as e:
        api.apply(L.OP_COPY, [x, x], shapes=[(64,), (64,)], counter=(32,), bases=[0, 16],
                  params=L.CopyParams(4))
    assert e.value.status == L.E_ALIAS


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6])
def test_embed_fill_matches_oracle(d):
    shapes = inputs.cfg4_shapes(n_pairs=64)
    sx, sy = [p for p in shapes if len(p[0]) == d][0]
    dst_s = inputs.padded_shape(sx, sy)
    announce("embed_fill", sx, dst_s)
    x = inputs.rng(4, 50, d).standard_normal(sx).astype(np.float32)
    want = np.full(dst_s, 9.0, dtype=np.float32)
    oracle.embed_fill(dst_s, want.reshape(-1), dst_s, x.reshape(-1), sx)
    got = host(api.pad_embed(dev(x), dst_s))
    assert bits_equal(got, want), first_mismatch(got, want)


def test_embed_fill_float64_and_window():
    announce("embed_fill f64 window")
    rng = np.random.default_rng(8)
    parent = (12, 15)
    src = rng.standard_normal(parent)
    base = 3 * 15 + 4                 # window starting at (3, 4): extents (9, 11)
    dst_s = (10, 14)
    want = np.zeros(dst_s)
    oracle.embed_fill(dst_s, want.reshape(-1), dst_s, src.reshape(-1), parent, 0, base)
    g = torch.empty(dst_s, dtype=torch.float64, device="cuda")
    api.embed_fill_(g, dev(src), src_base=base)
    got = host(g)
    assert bits_equal(got, want), first_mismatch(got, want)


# ---------------------------------------------------------------------------
# Element-wise products
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("d", range(2, 9))
@pytest.mark.parametrize("log2n", [12, 17])
def test_mul_acc_sweep_bit_exact(d, log2n):
    xs, ys, zs = inputs.cfg2_inter_shapes(d, log2_target=log2n)
    announce("mul_acc", d, xs, ys, zs)
    x = inputs.uniform(2, xs, 40, d, log2n)
    y = inputs.uniform(2, ys, 41, d, log2n)
    z = inputs.uniform(2, zs, 42, d, log2n)
    want = x.copy()
    oracle.mul_acc(xs, want.reshape(-1), xs, y.reshape(-1), ys, z.reshape(-1), zs)
    gx = dev(x)
    api.mul_acc_(gx, dev(y), dev(z))
    got = host(gx)
    assert bits_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("d", [2, 3, 4, 5])
def test_mul_acc_literal_intersection(d):
    a, b, c = inputs.cfg2_inter_literal_shapes(d, log2_target=13)
    counter = tuple(min(p, q, r) for p, q, r in zip(a, b, c))
    announce("mul_acc literal", d, a, b, c)
    x = inputs.uniform(2, a, 60, d)
    y = inputs.rng(2, 61, d).standard_normal(b).astype(np.float32)
    z = inputs.rng(2, 62, d).standard_normal(c).astype(np.float32)
    want = x.copy()
    oracle.mul_acc(counter, want.reshape(-1), a, y.reshape(-1), b, z.reshape(-1), c)
    gx = dev(x)
    api.mul_acc_(gx, dev(y), dev(z))
    got = host(gx)
    assert bits_equal(got, want), first_mismatch(got, want)


def test_mul_acc_rounding_denormals_and_aliasing():
    announce("mul_acc rounding")
    e = np.float32(2.0 ** -12)
    x = np.array([-(1 + 2 * e), 1e-38, 0.0, -0.0], dtype=np.float32)
    y = np.array([1 + e, 1e-3, 1e-30, 0.0], dtype=np.float32)
    z = np.array([1 + e, 1e-5, 1e-15, 1.0], dtype=np.float32)
    want = x.copy()
    oracle.mul_acc((4,), want, (4,), y, (4,), z, (4,))
    assert want[0] == 0.0                       # a fused multiply-add would give 2^-24
    gx = dev(x)
    api.mul_acc_(gx, dev(y), dev(z))
    got = host(gx)
    assert bits_equal(got, want), (got, want)
    # x[t] += y[t] * x[t] with x passed twice
    rng = np.random.default_rng(3)
    x = rng.standard_normal((37, 41)).astype(np.float32)
    y = rng.standard_normal((40, 45)).astype(np.float32)
    want = x.copy()
    oracle.mul_acc(x.shape, want.reshape(-1), x.shape, y.reshape(-1), y.shape, want.reshape(-1),
                   x.shape)
    gx = dev(x)
    api.mul_acc_(gx, dev(y), gx)
    got = host(gx)
    assert bits_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("shapes", [((28, 30, 32, 26, 32), (32,) * 5, (28, 30, 32, 26, 32)),
                                    ((5, 7, 3), (9, 7, 4), (6, 8, 3)),
                                    ((100, 3), (101, 5), (100, 4))])
def test_mul_bit_exact(shapes):
    os_, as_, bs = shapes
    announce("mul", shapes)
    a = inputs.rng(5, 70).standard_normal(as_).astype(np.float32)
    b = inputs.rng(5, 71).standard_normal(bs).astype(np.float32)
    want = np.zeros(os_, dtype=np.float32)
    oracle.mul(os_, want.reshape(-1), os_, a.reshape(-1), as_, b.reshape(-1), bs)
    got = host(api.mul(dev(a), dev(b), counter=os_))
    assert bits_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("shapes", [((32,) * 5, (28, 30, 32, 26, 32), (28, 30, 32, 26, 32)),
                                    ((9, 8, 7), (6, 9, 7), (5, 7, 6)),
                                    ((64, 65), (70, 33), (60, 30))])
def test_mul_adj_bit_exact(shapes):
    sa, sb, si = shapes
    announce("mul_adj", shapes)
    a = inputs.rng(5, 80).standard_normal(sa).astype(np.float32)
    b = inputs.rng(5, 81).standard_normal(sb).astype(np.float32)
    g = inputs.rng(5, 82).standard_normal(si).astype(np.float32)
    wa = np.full(sa, 5.0, dtype=np.float32)
    wb = np.full(sb, 5.0, dtype=np.float32)
    oracle.mul_adj(wa.reshape(-1), sa, wb.reshape(-1), sb, g.reshape(-1), si, a.reshape(-1),
                   b.reshape(-1))
    ga, gb = api.mul_adj(dev(g), dev(a), dev(b))
    ga, gb = host(ga), host(gb)
    assert bits_equal(ga, wa), first_mismatch(ga, wa)
    assert bits_equal(gb, wb), first_mismatch(gb, wb)


# ---------------------------------------------------------------------------
# Moments
# ---------------------------------------------------------------------------

def _check_moments(got32, got64, want, d, cov, tol=1e-6):
    n = 1 + d + (d * (d + 1) // 2 if cov else 0)
    want = want[:n]
    if cov and d:
        # entries whose exact value is 0 (e.g. independent axes) are judged
        # against the scale of the covariance diagonal
        diag = [want[1 + d + i * d - i * (i - 1) // 2] for i in range(d)]
        floor = 1e-6 * max(1.0, max(abs(v) for v in diag))
    else:
        floor = 0.0
    err32 = rel_err(got32[:n], want, floor=0.0)
    absok = np.abs(got32[:n].astype(np.float64) - want) <= tol * floor
    bad = ~((err32 <= tol) | absok)
    assert not bad.any(), ("float32 moments off", np.nonzero(bad)[0], got32[:n][bad], want[bad],
                           err32[bad])
    err64 = rel_err(got64[:n], want)
    absok64 = np.abs(got64[:n] - want) <= 1e-3 * tol * max(floor, 1e-300)
    assert ((err64 <= 1e-9) | absok64).all(), ("float64 moments off", err64.max())
    return float(err32[np.isfinite(err32)].max()) if n else 0.0


def test_moments_cfg3_full_size():
    announce("moments cfg3")
    p = inputs.cfg3_values()
    shape = inputs.CFG3_SHAPE
    want = oracle.moments(shape, [p.reshape(-1)], [shape], cov=True)
    o32, o64 = api.moments(dev(p), cov=True)
    g32 = host(o32)
    # the error of every one of the 28 results, reported before the check
    names = ["M"] + ["E%d" % i for i in range(6)] + ["C%d%d" % (i, j) for i in range(6)
                                                    for j in range(i, 6)]
    per = {nm: abs(float(g) - w) / abs(w) for nm, g, w in zip(names, g32, want)}
    print("cfg3 per-result relative error of the float32 results:",
          " ".join("%s=%.2e" % kv for kv in per.items()), flush=True)
    e = _check_moments(g32, host(o64), want, 6, True)
    print("cfg3 max relative error (float32 results):", e)


@pytest.mark.parametrize("shape", [(5,), (7, 3), (33, 17), (3, 64, 5), (100, 70), (2, 3, 4, 5, 6),
                                   (9, 5, 1, 7), (4, 1, 1, 3, 5, 2, 3, 2), (1000,), (3, 1000),
                                   (2, 2, 2, 2, 2, 2, 2, 2)])
@pytest.mark.parametrize("cov", [False, True])
def test_moments_shapes(shape, cov):
    announce("moments", shape, cov)
    rng = inputs.rng(3, 10, len(shape), int(np.prod(shape)))
    p = rng.gamma(0.5, 1.0, size=shape).astype(np.float32)
    want = oracle.moments(shape, [p.reshape(-1)], [shape], cov=cov)
    o32, o64 = api.moments(dev(p), cov=cov)
    _check_moments(host(o32), host(o64), want, len(shape), cov)
    # the cached-load hint changes how the operand is loaded, not the sums
    c32, c64 = api.moments(dev(p), cov=cov, cached=True)
    assert bits_equal(host(c32), host(o32)) and bits_equal(host(c64), host(o64))


# Rows of 4, 8 or 16 words laid end to end: segment counts below one wave,
# between waves and over several tiles, with dropped axes, one and several
# operands and both load hints.  The inner product takes its staged tile
# loads here (each wave loads its 64 segments line by line through LDS).
STAGED_SHAPES = [(7, 5, 16), (33, 29, 16), (300, 8), (5, 77, 4), (2, 3, 1, 4, 3, 8), (16,),
                 (3, 1, 257, 4), (64, 16), (65, 8, 16)]


@pytest.mark.parametrize("shape", STAGED_SHAPES)
@pytest.mark.parametrize("cov", [False, True])
def test_moments_short_rows(shape, cov):
    announce("moments short rows", shape, cov)
    rng = inputs.rng(3, 20, len(shape), int(np.prod(shape)))
    p = rng.gamma(0.5, 1.0, size=shape).astype(np.float32)
    q = rng.random(shape).astype(np.float32)
    d = len(shape)
    want = oracle.moments(shape, [p.reshape(-1)], [shape], cov=cov)
    for cached in (False, True):
        o32, o64 = api.moments(dev(p), cov=cov, cached=cached)
        _check_moments(host(o32), host(o64), want, d, cov)
    # two operands: w = p * q per point, formed in float64
    want2 = oracle.moments(shape, [p.reshape(-1), q.reshape(-1)], [shape, shape], cov=cov)
    o32, o64 = api.moments(dev(p), cov=cov, others=[dev(q)])
    _check_moments(host(o32), host(o64), want2, d, cov)


# Rows of 16 words laid end to end from 2^21 rows on: one operand takes the
# quads of 16-word rows (4 workgroups per CU), two operands the staged tile
# loads (3 per CU; just below 2^21 rows, per-lane loads).
@pytest.mark.parametrize("shape", [(2048, 1024, 16), (2047, 1024, 16), (8192, 257, 16)])
def test_moments_large_staged(shape):
    announce("moments large staged", shape)
    rng = inputs.rng(3, 25, shape[0], shape[1])
    p = rng.random(shape, dtype=np.float32)
    d = len(shape)
    for cov in (True, False):
        want = oracle.moments(shape, [p.reshape(-1)], [shape], cov=cov)
        o32, o64 = api.moments(dev(p), cov=cov)
        _check_moments(host(o32), host(o64), want, d, cov)
    if shape[0] == 2048:
        q = rng.random(shape, dtype=np.float32)
        want = oracle.moments(shape, [p.reshape(-1), q.reshape(-1)], [shape, shape], cov=True)
        o32, o64 = api.moments(dev(p), cov=True, others=[dev(q)])
        _check_moments(host(o32), host(o64), want, d, True)


# Rows of 16 words laid end to end, one operand: every load instruction
# covers 16 consecutive rows and the row sums are formed across the lanes of
# a quad.  Row counts that end the last wave after 1, 15, 17 or 63 of its 64
# rows, several tiles, both accumulator tiers (10 axes: first moments only)
# and both load hints.
@pytest.mark.parametrize("shape", [(1, 16), (17, 16), (63, 16), (1041, 16), (3, 5, 67, 16),
                                   (2, 3, 5, 7, 16), (2,) * 9 + (16,), (4099, 3, 16)])
def test_moments_row_quads(shape):
    announce("moments row quads", shape)
    rng = inputs.rng(3, 27, len(shape), int(np.prod(shape)))
    p = rng.gamma(0.5, 1.0, size=shape).astype(np.float32)
    d = len(shape)
    for cov in ((True, False) if d <= 8 else (False,)):
        want = oracle.moments(shape, [p.reshape(-1)], [shape], cov=cov)
        for cached in (False, True):
            o32, o64 = api.moments(dev(p), cov=cov, cached=cached)
            _check_moments(host(o32), host(o64), want, d, cov)


# Rows a multiple of 32 words laid end to end: the moments pass stages both
# halves of every 32-word segment (one operand); segment counts below one
# wave and ragged over several tiles; two operands keep per-lane loads.
@pytest.mark.parametrize("shape", [(5, 32), (33, 7, 64), (256, 256), (3, 5, 7, 96), (64, 64, 64),
                                   (1, 9, 1, 32)])
def test_moments_32_word_segments(shape):
    announce("moments 32-word segments", shape)
    rng = inputs.rng(3, 28, len(shape), int(np.prod(shape)))
    p = rng.gamma(0.5, 1.0, size=shape).astype(np.float32)
    d = len(shape)
    for cov in (True, False):
        want = oracle.moments(shape, [p.reshape(-1)], [shape], cov=cov)
        for cached in (False, True):
            o32, o64 = api.moments(dev(p), cov=cov, cached=cached)
            _check_moments(host(o32), host(o64), want, d, cov)
    q = rng.random(shape, dtype=np.float32)
    want = oracle.moments(shape, [p.reshape(-1), q.reshape(-1)], [shape, shape], cov=True)
    o32, o64 = api.moments(dev(p), cov=True, others=[dev(q)])
    _check_moments(host(o32), host(o64), want, d, True)


# Rows of at most 8 words, one operand: the moments pass loads the segments
# of several tiles before folding them.  Many small axes (both accumulator
# tiers), an inner extent that is not whole quads, and a window.
# (Rows of 2, 4 or 8 words laid end to end whose next axis is a multiple of
# 16 / L take 16-word row blocks instead: 4^12, 8^8, (3, 16, 2), (5, 12, 4),
# (7, 6, 8), (16^5, 4, 4).)
@pytest.mark.parametrize("shape,cov", [((4,) * 12, False), ((8,) * 8, True), ((3, 1000, 3), True),
                                       ((6, 5, 7, 6, 5, 7), True), ((2,) * 20, False),
                                       ((3, 16, 2), True), ((5, 12, 4), True), ((7, 6, 8), True),
                                       ((16, 16, 16, 16, 16, 4, 4), True), ((4,) * 8, False),
                                       ((9, 7, 8), True)])
def test_moments_short_rows_batched(shape, cov):
    announce("moments short rows batched", shape, cov)
    rng = inputs.rng(3, 30, len(shape), int(np.prod(shape)))
    p = rng.random(shape, dtype=np.float32)
    d = len(shape)
    want = oracle.moments(shape, [p.reshape(-1)], [shape], cov=cov)
    for cached in (False, True):
        o32, o64 = api.moments(dev(p), cov=cov, cached=cached)
        _check_moments(host(o32), host(o64), want, d, cov)


def test_moments_short_rows_window():
    announce("moments short rows window")
    rng = inputs.rng(3, 31)
    parent = (40, 50, 9)
    P = rng.random(parent, dtype=np.float32)
    base = int(np.ravel_multi_index((3, 2, 1), parent))
    counter = (33, 47, 7)
    want = oracle.moments(counter, [P.reshape(-1)], [parent], bases=[base])
    out32 = torch.empty(1 + 3 + 6, device="cuda")
    out64 = torch.empty(1 + 3 + 6, dtype=torch.float64, device="cuda")
    ws = api.workspace_for(L.OP_MOMENTS, [parent], counter, torch.device("cuda"))
    params = L.MomentsParams(L.MOMENTS_FIRST | L.MOMENTS_COV, out64.data_ptr())
    api.apply(L.OP_MOMENTS, [dev(P)], [parent], counter, [base], params, out=out32, workspace=ws)
    _check_moments(host(out32), host(out64), want, 3, True)


@pytest.mark.parametrize("shape", STAGED_SHAPES)
def test_dot_staged_rows(shape):
    announce("dot staged", shape)
    rng = inputs.rng(3, 21, len(shape), int(np.prod(shape)))
    a = rng.standard_normal(shape).astype(np.float32)
    b = rng.standard_normal(shape).astype(np.float32)
    c = rng.standard_normal(shape).astype(np.float32)
    n = int(np.prod(shape))
    for ops in ([a, b], [a, b, c], [a, b, c, a]):
        want = oracle.dot(shape, ops, [shape] * len(ops))
        mag = oracle.dot(shape, [np.abs(x) for x in ops], [shape] * len(ops))
        o32, o64 = api.dot(*[dev(x) for x in ops])
        g = float(host(o64)[0])
        # float64 sums in another order: within n eps sum|w| of the oracle
        assert abs(g - want) <= n * np.finfo(np.float64).eps * mag + 1e-300, (g, want)
    # integer values: exact whatever the order
    ai = rng.integers(-3, 4, size=shape).astype(np.float32)
    bi = rng.integers(-3, 4, size=shape).astype(np.float32)
    want = oracle.dot(shape, [ai, bi], [shape, shape])
    o32, o64 = api.dot(dev(ai), dev(bi))
    assert host(o64)[0] == want
    ci = rng.integers(-2, 3, size=shape).astype(np.float32)
    want = oracle.dot(shape, [ai, bi, ci, ai], [shape] * 4)
    o32, o64 = api.dot(dev(ai), dev(bi), dev(ci), dev(ai))
    assert host(o64)[0] == want


# Windows whose rows are whole word quads (the inner product's quad walk:
# one quad per lane): inner extents 4 .. 100, ragged last tiles, two and
# three operands, and a single long row.
QUAD_CASES = [((37, 41, 32), (40, 39, 36)), ((9, 10, 8), (12, 9, 8)), ((50, 12), (51, 13)),
              ((3, 7, 5, 64), (4, 7, 6, 66)), ((300, 100), (301, 104)), ((70000,), (65540,)),
              ((2, 1, 33, 4), (3, 1, 34, 4))]


@pytest.mark.parametrize("case", range(len(QUAD_CASES)))
def test_dot_quad_walk(case):
    sa, sb = QUAD_CASES[case]
    announce("dot quads", sa, sb)
    rng = inputs.rng(3, 24, case)
    a = rng.standard_normal(sa).astype(np.float32)
    b = rng.standard_normal(sb).astype(np.float32)
    counter = tuple(min(x, y) for x, y in zip(sa, sb))
    n = int(np.prod(counter))
    for ops, shapes in (([a, b], [sa, sb]), ([a, b, b], [sa, sb, sb])):
        want = oracle.dot(counter, ops, shapes)
        mag = oracle.dot(counter, [np.abs(x) for x in ops], shapes)
        o32, o64 = api.dot(*[dev(x) for x in ops])
        g = float(host(o64)[0])
        assert abs(g - want) <= n * np.finfo(np.float64).eps * mag + 1e-300, (g, want)
    ai = rng.integers(-3, 4, size=sa).astype(np.float32)
    bi = rng.integers(-3, 4, size=sb).astype(np.float32)
    want = oracle.dot(counter, [ai, bi], [sa, sb])
    o32, o64 = api.dot(dev(ai), dev(bi))
    assert host(o64)[0] == want
    # four operands over different windows (the intersection stays the
    # counter), integer values: exact whatever the order
    sc = tuple(x + 1 for x in counter)
    sd = tuple(x + 4 for x in counter)
    ci = rng.integers(-2, 3, size=sc).astype(np.float32)
    di = rng.integers(-2, 3, size=sd).astype(np.float32)
    want = oracle.dot(counter, [ai, bi, ci, di], [sa, sb, sc, sd])
    o32, o64 = api.dot(dev(ai), dev(bi), dev(ci), dev(di))
    assert host(o64)[0] == want


def test_moments_invariants_on_gpu():
    announce("moments invariants")
    # delta: E = t exactly
    shape = (16,) * 6
    p = np.zeros(shape, dtype=np.float32)
    t = (3, 15, 0, 7, 9, 1)
    p[t] = 1.0
    o32, o64 = api.moments(dev(p), cov=True)
    o64 = host(o64)
    assert list(o64[1:7]) == list(t)
    assert (o64[7:] == 0).all()
    # uniform: E = (s-1)/2, Var = (s^2-1)/12
    shape = (5, 8, 3, 6)
    o32, o64 = api.moments(torch.ones(shape, device="cuda"), cov=True)
    o64 = host(o64)
    s = np.asarray(shape, dtype=np.float64)
    assert np.allclose(o64[1:5], (s - 1) / 2, rtol=0, atol=1e-12)
    diag = [o64[5 + i * 4 - i * (i - 1) // 2] for i in range(4)]
    assert np.allclose(diag, (s * s - 1) / 12, rtol=1e-12)


def test_moments_several_operands_and_windows():
    announce("moments operands/windows")
    rng = np.random.default_rng(44)
    # w = x*y*z over the intersection (Algorithm 11's three-tensor form)
    xs, ys, zs = (20, 30, 10), (25, 30, 12), (20, 31, 10)
    x, y, z = (rng.random(s).astype(np.float32) for s in (xs, ys, zs))
    counter = (20, 30, 10)
    want = oracle.moments(counter, [x.reshape(-1), y.reshape(-1), z.reshape(-1)], [xs, ys, zs])
    o32, o64 = api.moments(dev(x), cov=True, others=[dev(y), dev(z)])
    # the float32 product of three weights is rounded once per point, so
    # the float64 results carry that rounding (relative 2^-23 per point)
    got = host(o64)
    err = rel_err(got, want, floor=1e-6 * abs(want[4]))
    assert err.max() <= 1e-6, err
    # a window (non-contiguous operand): the per-thread path
    parent = (40, 50, 30)
    P = rng.random(parent).astype(np.float32)
    base = int(np.ravel_multi_index((3, 7, 2), parent))
    counter = (20, 30, 25)
    want = oracle.moments(counter, [P.reshape(-1)], [parent], bases=[base])
    out32 = torch.empty(1 + 3 + 6, device="cuda")
    out64 = torch.empty(1 + 3 + 6, dtype=torch.float64, device="cuda")
    ws = api.workspace_for(L.OP_MOMENTS, [parent], counter, torch.device("cuda"))
    params = L.MomentsParams(L.MOMENTS_FIRST | L.MOMENTS_COV, out64.data_ptr())
    api.apply(L.OP_MOMENTS, [dev(P)], [parent], counter, [base], params, out=out32, workspace=ws)
    _check_moments(host(out32), host(out64), want, 3, True)


def test_moments_first_high_dimension():
    shape = (2, 3, 2, 2, 3, 2, 2, 2, 3, 2, 2, 2)
    announce("moments d12 first", shape)
    p = inputs.rng(3, 12).random(shape).astype(np.float32)
    want = oracle.moments(shape, [p.reshape(-1)], [shape], cov=False)
    o32, o64 = api.moments(dev(p), cov=False)
    _check_moments(host(o32), host(o64), want, len(shape), False)


def test_moments_zero_mass_and_scalar():
    announce("moments degenerate")
    o32, o64 = api.moments(torch.zeros((4, 4), device="cuda"), cov=True)
    o64 = host(o64)
    assert o64[0] == 0 and np.isnan(o64[1:]).all()
    o32, o64 = api.moments(torch.full((), 2.5, device="cuda"), cov=True)
    assert host(o64).tolist() == [2.5]


# ---------------------------------------------------------------------------
# Moments adjoint
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape,cov", [((16,) * 6, True), ((28, 30, 32, 26, 32), False),
                                       ((7, 1, 40), True), ((3, 100), True), ((2, 3, 2, 3, 2, 3, 2, 3, 2, 3), False)])
def test_moments_adj_matches_oracle(shape, cov):
    announce("moments_adj", shape, cov)
    d = len(shape)
    rng = inputs.rng(3, 30, d)
    nout = 1 + d + (d * (d + 1) // 2 if cov else 0)
    mom = rng.standard_normal(nout)
    mom[0] = abs(mom[0]) + 0.5
    mom[1:1 + d] = np.asarray(shape) / 2.0 + rng.standard_normal(d)
    gmom = rng.standard_normal(nout).astype(np.float32)
    want = np.zeros(shape)
    oracle.moments_adj(shape, want.reshape(-1), shape, mom, gmom.astype(np.float64), cov=cov)
    got = host(api.moments_adj(shape, dev(mom), dev(gmom), cov=cov))
    w32 = want.astype(np.float32)
    rms = float(np.sqrt(np.mean(want ** 2)))
    err = rel_err(got, want, floor=1e-3 * rms)
    assert err.max() <= 1e-6, (err.max(), np.unravel_index(err.argmax(), shape))
    # nearly always identical to the rounded float64 value
    assert np.mean(got == w32) > 0.99
