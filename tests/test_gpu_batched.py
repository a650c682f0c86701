"""The batched form: thousands of ragged items in one persistent launch,
captured in a hipGraph and replayed, against the oracle item by item."""
import numpy as np
import pytest
import torch

import oracle
from paper_1608_00099_amd import _lib as L
from paper_1608_00099_amd import api, inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu


def _check_items(dsts, xs_np, shapes):
    for i, (d_, x, (sx, sy)) in enumerate(zip(dsts, xs_np, shapes)):
        ps = inputs.padded_shape(sx, sy)
        want = np.full(ps, 3.0, dtype=np.float32)
        oracle.embed_fill(ps, want.reshape(-1), ps, x.reshape(-1), sx)
        got = d_.cpu().numpy()
        assert got.tobytes() == want.tobytes(), ("item", i, sx, sy)


def test_batched_fft_padding_full_4096_items():
    announce("batched cfg4 4096 items")
    shapes = inputs.cfg4_shapes()
    xs_np = inputs.cfg4_values(shapes)
    xs = [torch.from_numpy(x).cuda() for x in xs_np]
    dsts = [torch.full(inputs.padded_shape(sx, sy), 7.0, device="cuda") for sx, sy in shapes]
    items = [[d_, x] for d_, x in zip(dsts, xs)]
    b = api.Batch()
    b.apply(L.OP_EMBED_FILL, items)
    torch.cuda.synchronize()
    info = b.info()
    assert info["replayed"] is False and info["units"] > 0
    _check_items(dsts, xs_np, shapes)
    # replays of the captured graph, with eager work between them
    for rep in range(3):
        for d_ in dsts:
            d_.fill_(-1.0 - rep)
        torch.cuda.synchronize()
        if rep == 1:
            b.apply(L.OP_EMBED_FILL, items)       # re-validated replay
        else:
            b.launch()                            # plain replay
        torch.cuda.synchronize()
        assert b.info()["replayed"] is True
        _check_items(dsts, xs_np, shapes)
    b.close()


@pytest.mark.parametrize("order", [1, 0])
def test_batched_replan_and_other_ops(order):
    announce("batched mixed ops", order)
    rng = np.random.default_rng(9)
    b = api.Batch()
    if order != 1:
        b.set_schedule(unit_order=order)
    # MUL_ACC over intersections of ragged items of every d
    xs, ys, zs, want = [], [], [], []
    for d in range(1, 7):
        for k in range(5):
            x_s = tuple(int(v) for v in rng.integers(1, 20, size=d))
            y_s = tuple(s + int(rng.integers(0, 3)) for s in x_s)
            z_s = tuple(s + int(rng.integers(0, 3)) for s in x_s)
            x = rng.standard_normal(x_s).astype(np.float32)
            y = rng.standard_normal(y_s).astype(np.float32)
            z = rng.standard_normal(z_s).astype(np.float32)
            w = x.copy()
            oracle.mul_acc(x_s, w.reshape(-1), x_s, y.reshape(-1), y_s, z.reshape(-1), z_s)
            xs.append(torch.from_numpy(x).cuda())
            ys.append(torch.from_numpy(y).cuda())
            zs.append(torch.from_numpy(z).cuda())
            want.append(w)
    b.apply(L.OP_MUL_ACC, [[x, y, z] for x, y, z in zip(xs, ys, zs)])
    torch.cuda.synchronize()
    for x, w in zip(xs, want):
        assert x.cpu().numpy().tobytes() == w.tobytes()
    # a different batch on the same handle re-plans (COPY, 8-byte elements)
    srcs = [torch.from_numpy(rng.standard_normal((4, 5, 6))).cuda() for _ in range(7)]
    dsts = [torch.zeros((6, 7, 9), dtype=torch.float64, device="cuda") for _ in range(7)]
    b.apply(L.OP_COPY, [[d_, s] for d_, s in zip(dsts, srcs)], elem_bytes=8)
    torch.cuda.synchronize()
    assert b.info()["replayed"] is False
    for d_, s in zip(dsts, srcs):
        w = np.zeros((6, 7, 9))
        sn = s.cpu().numpy()
        oracle.copy((4, 5, 6), w.reshape(-1), (6, 7, 9), sn.reshape(-1), (4, 5, 6))
        assert d_.cpu().numpy().tobytes() == w.tobytes()
    b.close()


def test_batched_empty_and_errors():
    announce("batched edge cases")
    b = api.Batch()
    # items with no points
    e1 = torch.zeros((3, 0), device="cuda")
    e2 = torch.zeros((3, 0), device="cuda")
    b.apply(L.OP_COPY, [[e1, e2]])
    assert b.info()["units"] == 0
    b.launch()
    # an invalid item reports its status and leaves the handle usable
    a = torch.zeros((4, 4), device="cuda")
    c = torch.zeros((3, 5), device="cuda")
    with pytest.raises(L.TriotError) as e:
        st = L.triot_apply_batched(L.OP_COPY, [(2, 2, [(4, 4), (3, 5)], (4, 4),
                                                 [a.data_ptr(), c.data_ptr()], None)],
                                   L.CopyParams(4), b._h, torch.cuda.current_stream().cuda_stream)
        api._check(st, "apply_batched")
    assert e.value.status == L.E_BOUNDS
    with pytest.raises(L.TriotError):
        api._check(L.triot_apply_batched(L.OP_MOMENTS, [], None, b._h, 0), "apply_batched")
    b.close()


@pytest.mark.parametrize("cache,bpc,unit,order", [(0, 4, 4096, 0), (1, 4, 4096, 0), (2, 2, 64, 0),
                                                  (0, 8, 1 << 16, 0), (1, 1, 1024, 0),
                                                  (1, 1, 4096, 1), (1, 8, 4096, 1), (2, 2, 64, 1),
                                                  (0, 4, 1 << 16, 1)])
def test_batched_schedules(cache, bpc, unit, order):
    """Every schedule gives the oracle's bits; unit order 1 deals the work
    units of all items round-robin over the workgroups."""
    announce("batched schedule cache=%d bpc=%d unit=%d order=%d" % (cache, bpc, unit, order))
    shapes = inputs.cfg4_shapes()[:300]
    xs_np = inputs.cfg4_values(shapes)
    xs = [torch.from_numpy(x).cuda() for x in xs_np]
    dsts = [torch.full(inputs.padded_shape(sx, sy), 7.0, device="cuda") for sx, sy in shapes]
    b = api.Batch()
    b.set_schedule(cache_policy=cache, blocks_per_cu=bpc, unit_elems=unit, unit_order=order)
    b.apply(L.OP_EMBED_FILL, [[d_, x] for d_, x in zip(dsts, xs)])
    torch.cuda.synchronize()
    _check_items(dsts, xs_np, shapes)
    for d_ in dsts:
        d_.fill_(-2.0)
    b.launch()
    torch.cuda.synchronize()
    _check_items(dsts, xs_np, shapes)
    # a new schedule drops the captured graph: replay needs a new apply
    b.set_schedule(cache_policy=(cache + 1) % 3, blocks_per_cu=bpc, unit_elems=unit,
                   unit_order=1 - order)
    with pytest.raises(L.TriotError):
        b.launch()
    for d_ in dsts:
        d_.fill_(5.0)
    b.apply(L.OP_EMBED_FILL, [[d_, x] for d_, x in zip(dsts, xs)])
    torch.cuda.synchronize()
    assert b.info()["replayed"] is False
    _check_items(dsts, xs_np, shapes)
    b.close()


def test_batched_schedule_rejects_out_of_range():
    announce("batched schedule errors")
    b = api.Batch()
    for kw in ({"cache_policy": 3}, {"blocks_per_cu": 0}, {"blocks_per_cu": 33},
               {"unit_elems": 63}, {"box_rows_max": 0}, {"unit_order": 2}):
        with pytest.raises(L.TriotError) as e:
            b.set_schedule(**kw)
        assert e.value.status == L.E_INVALID
    b.close()


def test_batched_lane_widths_agree():
    """Items with 4-word lanes (the default) and with 1-word lanes give the
    oracle's bits, EMBED_FILL and MUL_ACC."""
    announce("batched lane widths")
    shapes = inputs.cfg4_shapes()[300:700]
    xs_np = inputs.cfg4_values(shapes)
    xs = [torch.from_numpy(x).cuda() for x in xs_np]
    for vec in (4, 1):
        dsts = [torch.full(inputs.padded_shape(sx, sy), 7.0, device="cuda") for sx, sy in shapes]
        b = api.Batch()
        b.set_schedule(vec_max=vec)
        b.apply(L.OP_EMBED_FILL, [[d_, x] for d_, x in zip(dsts, xs)])
        torch.cuda.synchronize()
        _check_items(dsts, xs_np, shapes)
        b.close()
    rng = np.random.default_rng(31)
    for vec in (4, 1):
        b = api.Batch()
        b.set_schedule(vec_max=vec)
        items, want = [], []
        for k in range(40):
            d = 1 + k % 4
            x_s = tuple(int(v) for v in rng.integers(3, 40, size=d))
            y_s = tuple(s + int(rng.integers(0, 3)) for s in x_s)
            x = rng.standard_normal(x_s).astype(np.float32)
            y = rng.standard_normal(y_s).astype(np.float32)
            z = rng.standard_normal(y_s).astype(np.float32)
            w = x.copy()
            oracle.mul_acc(x_s, w.reshape(-1), x_s, y.reshape(-1), y_s, z.reshape(-1), y_s)
            items.append([torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda(),
                          torch.from_numpy(z).cuda()])
            want.append(w)
        b.apply(L.OP_MUL_ACC, items)
        torch.cuda.synchronize()
        for it, w in zip(items, want):
            assert it[0].cpu().numpy().tobytes() == w.tobytes()
        b.close()


@pytest.mark.parametrize("bpc,unit", [(1, 64), (2, 256)])
def test_batched_uneven_items_round_robin(bpc, unit):
    """One large item among many tiny ones, units dealt round-robin: each
    workgroup's consecutive units fall in items far apart, found by binary
    search over the items' first units."""
    announce("batched uneven items", bpc, unit)
    rng = np.random.default_rng(77 + bpc)
    shapes = [((1024, 1000), (700, 900))]
    for k in range(300):
        d = 1 + k % 3
        dst_s = tuple(int(v) for v in rng.integers(1, 12, size=d))
        src_s = tuple(int(rng.integers(1, s + 1)) for s in dst_s)
        shapes.append((dst_s, src_s))
    shapes.insert(150, ((33, 47, 29), (20, 40, 29)))
    xs_np = [rng.standard_normal(sx).astype(np.float32) for _, sx in shapes]
    dsts = [torch.full(ds, 7.0, device="cuda") for ds, _ in shapes]
    xs = [torch.from_numpy(x).cuda() for x in xs_np]
    b = api.Batch()
    b.set_schedule(blocks_per_cu=bpc, unit_elems=unit, unit_order=1)
    b.apply(L.OP_EMBED_FILL, [[d_, x] for d_, x in zip(dsts, xs)])
    torch.cuda.synchronize()
    assert b.info()["units"] > b.info()["blocks"]
    for i, (d_, x, (ds, sx)) in enumerate(zip(dsts, xs_np, shapes)):
        want = np.full(ds, 7.0, dtype=np.float32)
        oracle.embed_fill(ds, want.reshape(-1), ds, x.reshape(-1), sx)
        got = d_.cpu().numpy()
        assert got.tobytes() == want.tobytes(), ("item", i, ds, sx)
    b.close()


def test_batched_overlapping_items_rejected_nothing_enqueued():
    announce("batched cross-item overlap")
    a = torch.full((64,), 5.0, device="cuda")
    src = torch.arange(64, dtype=torch.float32, device="cuda")
    b = api.Batch()
    # a valid batch is planned first: a rejected call must leave it usable
    b.apply(L.OP_COPY, [[a[:32], src[:32]]])
    torch.cuda.synchronize()
    assert torch.equal(a[:32], src[:32]) and bool((a[32:] == 5.0).all())
    a.fill_(5.0)
    torch.cuda.synchronize()
    # item 1 writes into what item 0 reads (a window of one parent buffer)
    st = L.triot_apply_batched(
        L.OP_COPY,
        [(1, 2, [(16,), (64,)], (16,), [a.data_ptr(), src.data_ptr()], [0, 8]),
         (1, 2, [(16,), (16,)], None, [src.data_ptr() + 4 * 16, a.data_ptr() + 4 * 32], None)],
        L.CopyParams(4), b._h, torch.cuda.current_stream().cuda_stream)
    assert st == L.E_ALIAS
    with pytest.raises(L.TriotError) as e:
        b.autotune(L.OP_COPY, [[a[:32], src[:32]], [src[16:48], a[32:]]])
    assert e.value.status == L.E_ALIAS
    torch.cuda.synchronize()
    assert bool((a == 5.0).all())
    assert torch.equal(src, torch.arange(64, dtype=torch.float32, device="cuda"))
    # the earlier plan still replays
    b.launch()
    torch.cuda.synchronize()
    assert torch.equal(a[:32], src[:32])
    b.close()


def test_batched_autotune_cfg4_bit_exact():
    announce("batched autotune cfg4 4096 items")
    shapes = inputs.cfg4_shapes()
    xs_np = inputs.cfg4_values(shapes)
    xs = [torch.from_numpy(x).cuda() for x in xs_np]
    dsts = [torch.full(inputs.padded_shape(sx, sy), 7.0, device="cuda") for sx, sy in shapes]
    items = [[d_, x] for d_, x in zip(dsts, xs)]
    b = api.Batch()
    default = b.schedule()
    b.autotune(L.OP_EMBED_FILL, items)
    tuned = b.schedule()
    print("default", default, "tuned", tuned)
    for d_ in dsts:
        d_.fill_(-2.0)
    torch.cuda.synchronize()
    b.apply(L.OP_EMBED_FILL, items)
    torch.cuda.synchronize()
    assert b.info()["replayed"] is False
    _check_items(dsts, xs_np, shapes)
    # a second handle over new buffers of the same layout picks up the tuned
    # schedule (same launch grid) and gives the same bits
    dsts2 = [torch.full(inputs.padded_shape(sx, sy), 9.0, device="cuda") for sx, sy in shapes]
    b2 = api.Batch()
    b2.apply(L.OP_EMBED_FILL, [[d_, x] for d_, x in zip(dsts2, xs)])
    torch.cuda.synchronize()
    assert b2.info()["blocks"] == b.info()["blocks"]
    assert b2.info()["units"] == b.info()["units"]
    _check_items(dsts2, xs_np, shapes)
    b.close()
    b2.close()
    api.tune_reset()


def test_batched_autotune_mul_acc_small():
    announce("batched autotune mul_acc")
    rng = np.random.default_rng(21)
    xs, ys, zs, x0 = [], [], [], []
    for d in range(1, 5):
        for k in range(6):
            x_s = tuple(int(v) for v in rng.integers(1, 40, size=d))
            y_s = tuple(s + int(rng.integers(0, 4)) for s in x_s)
            z_s = tuple(s + int(rng.integers(0, 4)) for s in x_s)
            x = rng.standard_normal(x_s).astype(np.float32)
            xs.append(torch.from_numpy(x).cuda())
            ys.append(torch.from_numpy(rng.standard_normal(y_s).astype(np.float32)).cuda())
            zs.append(torch.from_numpy(rng.standard_normal(z_s).astype(np.float32)).cuda())
            x0.append(x)
    items = [[x, y, z] for x, y, z in zip(xs, ys, zs)]
    b = api.Batch()
    b.autotune(L.OP_MUL_ACC, items)          # runs x += y*z several times
    for x, x_init in zip(xs, x0):
        x.copy_(torch.from_numpy(x_init))
    b.apply(L.OP_MUL_ACC, items)
    torch.cuda.synchronize()
    for x, y, z, x_init in zip(xs, ys, zs, x0):
        w = x_init.copy()
        yn, zn = y.cpu().numpy(), z.cpu().numpy()
        oracle.mul_acc(w.shape, w.reshape(-1), w.shape, yn.reshape(-1), yn.shape,
                       zn.reshape(-1), zn.shape)
        assert x.cpu().numpy().tobytes() == w.tobytes()
    b.close()
    api.tune_reset()
