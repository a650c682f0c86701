"""Vector lanes over ragged rows: an inner extent that is not a multiple of
the vector width.  Each row's last vector is moved back to end at the row
end; it reads words of the vector before it again and stores only its new
words (COPY stores it whole: the shared words get the same source words).
Every case runs the op with the vector width pinned and compares with the
CPU oracle bit for bit, including the in-place forms (an output passed
again as an input) where a stored shared word would be read twice."""
import numpy as np
import pytest
import torch

import oracle
from paper_1608_00099_amd import _lib as L
from paper_1608_00099_amd import api
from tests.gpu_util import announce, bits_equal, dev, first_mismatch, host

pytestmark = pytest.mark.gpu

# (counter, grow of the larger operands per axis, base shift of those in elements)
CASES = [
    ((17, 3), (2, 1), 1),
    ((11, 5), (1, 3), 2),
    ((9, 6), (0, 2), 3),
    ((7, 13, 7), (1, 2, 1), 0),
    ((33, 9), (3, 2), 5),
    ((3, 4, 5, 39), (1, 1, 3, 12), 7),
    ((21, 145), (2, 14), 1),
    ((2, 3, 1023), (0, 1, 5), 2),
    ((100003,), (5,), 3),
]

# (vec_max, cache_policy, box_rows_max, unit_elems)
SCHEDS = [(4, 1, 1024, 8192), (4, 0, 1, 256), (2, 2, 1024, 64), (4, 2, 7, 1000)]


@pytest.fixture(autouse=True)
def _reset():
    api.tune_reset()
    yield
    api.tune_reset()


def _pin(op, tensors, shapes, counter, sched, bases=None, params=None):
    v, c, r, p = sched
    api.schedule_set(op, tensors, shapes=shapes, counter=counter, bases=bases, params=params,
                     vec_max=v, cache_policy=c, blocks_per_cu=4, box_rows_max=r, unit_elems=p,
                     unit_order=0)
    plan = api.describe(op, shapes, counter=counter, ptrs=[t.data_ptr() for t in tensors],
                        bases=bases, params=params)
    inner = counter[-1]
    if inner % v:
        want_vec = v if inner > v else (2 if inner > 2 and v == 4 else 1)
    else:
        want_vec = v
    # (a ragged width needs inner > width; a whole width needs inner >= 2 widths)
    return plan, want_vec


def _shapes(counter, grow):
    return tuple(c + g for c, g in zip(counter, grow))


def _base(counter, shape, shift):
    """A window start (a, 0, ..., 0, b) in `shape`, flattened, with a and b
    the shift or the room the counter leaves on that axis if less."""
    t = [0] * len(shape)
    t[0] = min(shift, shape[0] - counter[0])
    t[-1] = min(shift, shape[-1] - counter[-1])
    f = 0
    for i, s in enumerate(shape):
        f = f * s + t[i]
    return f


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("case", range(len(CASES)))
def test_ragged_copy_and_mul_acc(case, sched):
    counter, grow, shift = CASES[case]
    big = _shapes(counter, grow)
    bb = _base(counter, big, shift)
    rng = np.random.default_rng(700 + case)
    announce("ragged copy", counter, big, bb, sched)
    src = rng.standard_normal(big).astype(np.float32)
    dst = np.full(big, 3.0, dtype=np.float32)
    want = dst.copy()
    oracle.copy(counter, want.reshape(-1), big, src.reshape(-1), big, bb, 0)
    g, gs = dev(dst), dev(src)
    plan, _ = _pin(L.OP_COPY, [g, gs], [big, big], counter, sched, bases=[bb, 0],
                   params=L.CopyParams(4))
    api.copy_(g, gs, counter=counter, dst_base=bb, src_base=0)
    assert bits_equal(host(g), want), first_mismatch(host(g), want)

    announce("ragged mul_acc", counter, big, bb, sched, plan["vec"], plan["row_tail"])
    x = rng.standard_normal(counter).astype(np.float32)
    y = rng.standard_normal(big).astype(np.float32)
    z = rng.standard_normal(big).astype(np.float32)
    want = x.copy()
    oracle.mul_acc(counter, want.reshape(-1), counter, y.reshape(-1), big, z.reshape(-1), big,
                   0, bb, 0)
    gx, gy, gz = dev(x), dev(y), dev(z)
    plan, want_vec = _pin(L.OP_MUL_ACC, [gx, gy, gz], [counter, big, big], counter, sched,
                          bases=[0, bb, 0])
    if counter[-1] > 2:
        assert plan["vec"] == want_vec, plan
    if plan["vec"] > 1:
        assert plan["row_tail"] == counter[-1] % plan["vec"], plan
    api.mul_acc_(gx, gy, gz, counter=counter, bases=[0, bb, 0])
    assert bits_equal(host(gx), want), first_mismatch(host(gx), want)

    announce("ragged mul_acc in place", counter, sched)
    want = x.copy()
    oracle.mul_acc(counter, want.reshape(-1), counter, y.reshape(-1), big, want.reshape(-1),
                   counter, 0, bb, 0)
    gx = dev(x)
    _pin(L.OP_MUL_ACC, [gx, gy, gx], [counter, big, counter], counter, sched, bases=[0, bb, 0])
    api.mul_acc_(gx, gy, gx, counter=counter, shapes=[counter, big, counter], bases=[0, bb, 0])
    assert bits_equal(host(gx), want), first_mismatch(host(gx), want)


@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("case", range(len(CASES)))
def test_ragged_mul_and_xpyx_mz(case, sched):
    counter, grow, shift = CASES[case]
    big = _shapes(counter, grow)
    rng = np.random.default_rng(800 + case)
    a = rng.standard_normal(big).astype(np.float32)
    b = rng.standard_normal(counter).astype(np.float32)
    announce("ragged mul", counter, big, sched)
    want = np.zeros(counter, dtype=np.float32)
    oracle.mul(counter, want.reshape(-1), counter, a.reshape(-1), big, b.reshape(-1), counter)
    out = torch.empty(counter, dtype=torch.float32, device="cuda")
    ga, gb = dev(a), dev(b)
    _pin(L.OP_MUL, [out, ga, gb], [counter, big, counter], counter, sched)
    api.mul_into(out, ga, gb, counter=counter)
    assert bits_equal(host(out), want), first_mismatch(host(out), want)

    announce("ragged mul in place", counter, sched)
    want = b.copy()
    oracle.mul(counter, want.reshape(-1), counter, a.reshape(-1), big, want.reshape(-1), counter)
    gb = dev(b)
    _pin(L.OP_MUL, [gb, ga, gb], [counter, big, counter], counter, sched)
    api.mul_into(gb, ga, gb, counter=counter)
    assert bits_equal(host(gb), want), first_mismatch(host(gb), want)

    announce("ragged xpyx_mz", counter, sched)
    x = rng.standard_normal(counter).astype(np.float32)
    z = rng.standard_normal(big).astype(np.float32)
    want = x.copy()
    oracle.xpyx_mz(counter, want.reshape(-1), counter, a.reshape(-1), big, z.reshape(-1), big)
    gx, gz = dev(x), dev(z)
    _pin(L.OP_XPYX_MZ, [gx, ga, gz], [counter, big, big], counter, sched)
    api.xpyx_mz_(gx, ga, gz, counter=counter)
    assert bits_equal(host(gx), want), first_mismatch(host(gx), want)


# EMBED_FILL over a destination counter: (dst shape, src shape, src base
# shift).  Ragged destination rows and source inner bounds at every
# residue mod 4, so vectors lie wholly inside, straddle or lie past the
# source window.
FILL_CASES = [
    ((9, 11), (7, 9), 0),
    ((13, 6), (13, 5), 0),
    ((5, 7, 23), (4, 7, 21), 0),
    ((6, 5, 4, 39), (3, 5, 4, 17), 0),
    ((3, 1030), (3, 1027), 0),
    ((2, 8, 16), (2, 8, 13), 0),
    ((40, 41), (40, 38), 1),
    ((100003,), (99998,), 2),
]


@pytest.mark.parametrize("vec", [4, 2, 1])
@pytest.mark.parametrize("case", range(len(FILL_CASES)))
def test_embed_fill_vectors_with_ragged_rows_and_bounds(case, vec):
    dst_s, src_s, shift = FILL_CASES[case]
    announce("fill vectors", dst_s, src_s, shift, vec)
    rng = np.random.default_rng(900 + case)
    # the source window: src_s inside a parent grown by `shift` on the last axis
    parent = tuple(src_s[:-1]) + (src_s[-1] + shift,)
    x = rng.standard_normal(parent).astype(np.float32)
    want = np.full(dst_s, 7.0, dtype=np.float32)
    oracle.embed_fill(dst_s, want.reshape(-1), dst_s, x.reshape(-1), parent, 0, shift)
    g = torch.full(dst_s, 7.0, dtype=torch.float32, device="cuda")
    gx = dev(x)
    shapes = [dst_s, parent]
    api.schedule_set(L.OP_EMBED_FILL, [g, gx], shapes=shapes, counter=dst_s, bases=[0, shift],
                     params=L.CopyParams(4), vec_max=vec, cache_policy=1, blocks_per_cu=4,
                     box_rows_max=1024, unit_elems=8192, unit_order=0)
    plan = api.describe(L.OP_EMBED_FILL, shapes, counter=dst_s, ptrs=[g.data_ptr(), gx.data_ptr()],
                        bases=[0, shift], params=L.CopyParams(4))
    if vec == 4 and dst_s[-1] > 4:
        assert plan["vec"] == 4
    api.apply(L.OP_EMBED_FILL, [g, gx], shapes, dst_s, [0, shift], L.CopyParams(4),
              what="embed_fill")
    assert bits_equal(host(g), want), first_mismatch(host(g), want)


# Short source rows (fewer elements than a vector) under vector lanes: the
# source is read word by word.
SHORT_FILL_CASES = [
    ((9, 11), (7, 3), 0),
    ((6, 9), (6, 1), 1),
    ((5, 14), (5, 2), 0),
    ((4, 3, 10), (4, 2, 3), 2),
]


@pytest.mark.parametrize("case", range(len(SHORT_FILL_CASES)))
def test_embed_fill_short_source_rows(case):
    dst_s, src_s, shift = SHORT_FILL_CASES[case]
    announce("fill short source rows", dst_s, src_s, shift)
    rng = np.random.default_rng(950 + case)
    parent = tuple(src_s[:-1]) + (src_s[-1] + shift,)
    x = rng.standard_normal(parent).astype(np.float32)
    want = np.full(dst_s, 7.0, dtype=np.float32)
    oracle.embed_fill(dst_s, want.reshape(-1), dst_s, x.reshape(-1), parent, 0, shift)
    g = torch.full(dst_s, 7.0, dtype=torch.float32, device="cuda")
    gx = dev(x)
    shapes = [dst_s, parent]
    plan = api.describe(L.OP_EMBED_FILL, shapes, counter=dst_s, ptrs=[g.data_ptr(), gx.data_ptr()],
                        bases=[0, shift], params=L.CopyParams(4))
    assert plan["vec"] == 4, plan
    api.apply(L.OP_EMBED_FILL, [g, gx], shapes, dst_s, [0, shift], L.CopyParams(4),
              what="embed_fill")
    assert bits_equal(host(g), want), first_mismatch(host(g), want)


# One row of 4190211 elements: 1047553 four-word vectors, the last ragged
# (3 words), in 1024 work units of 1024 vectors: the last unit holds only
# the ragged vector.  Sources of the fills end inside the first vector of a
# unit (element 4096 * 500 + 2) and inside the ragged vector.
ROW = 4190211


def _one_row_plan(op, tensors, shapes, params=None):
    plan = api.describe(op, shapes, ptrs=[t.data_ptr() for t in tensors], params=params)
    assert plan["vec"] == 4 and plan["row_tail"] == 3 and plan["units"] == 1024, plan
    assert plan["box_rows"] == 1, plan


def test_unit_starting_at_a_ragged_vector_or_a_straddle():
    rng = np.random.default_rng(990)
    announce("one-row copy, last unit = ragged vector", ROW)
    src = rng.standard_normal(ROW).astype(np.float32)
    dst = np.full(ROW, 3.0, dtype=np.float32)
    g, gs = dev(dst), dev(src)
    _one_row_plan(L.OP_COPY, [g, gs], [(ROW,), (ROW,)], L.CopyParams(4))
    api.copy_(g, gs)
    assert bits_equal(host(g), src), first_mismatch(host(g), src)

    announce("one-row mul_acc", ROW)
    y = rng.standard_normal(ROW).astype(np.float32)
    z = rng.standard_normal(ROW).astype(np.float32)
    want = src.copy()
    oracle.mul_acc((ROW,), want, (ROW,), y, (ROW,), z, (ROW,))
    gx, gy, gz = dev(src), dev(y), dev(z)
    _one_row_plan(L.OP_MUL_ACC, [gx, gy, gz], [(ROW,)] * 3)
    api.mul_acc_(gx, gy, gz)
    assert bits_equal(host(gx), want), first_mismatch(host(gx), want)

    for n_src in (4096 * 500 + 2, ROW - 1, ROW - 2):
        announce("one-row fill", ROW, n_src)
        x = rng.standard_normal(n_src).astype(np.float32)
        want = np.full(ROW, 7.0, dtype=np.float32)
        oracle.embed_fill((ROW,), want, (ROW,), x, (n_src,))
        g = torch.full((ROW,), 7.0, dtype=torch.float32, device="cuda")
        gx = dev(x)
        _one_row_plan(L.OP_EMBED_FILL, [g, gx], [(ROW,), (n_src,)], L.CopyParams(4))
        api.embed_fill_(g, gx)
        assert bits_equal(host(g), want), first_mismatch(host(g), want)
