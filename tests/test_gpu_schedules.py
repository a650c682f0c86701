"""Every launch schedule gives the oracle's bits: the schedule knobs (vector
width, cache policy, workgroups per CU, unit order, box rows, work-unit
size) change the speed of a co-iteration, never its result.  Each case pins
one schedule through triot_schedule_set, runs the op, and compares with the
CPU oracle bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from paper_1608_00099_amd import _lib as L
from paper_1608_00099_amd import api, inputs
from tests.gpu_util import announce, bits_equal, dev, first_mismatch, host

pytestmark = pytest.mark.gpu

# (vec_max, cache_policy, blocks_per_cu, box_rows_max, unit_elems, unit_order)
SCHEDULES = [
    (4, 0, 4, 1024, 8192, 0),
    (4, 1, 4, 1024, 8192, 1),
    (4, 2, 4, 1024, 8192, 0),
    (2, 1, 1, 1024, 8192, 1),
    (1, 0, 2, 1024, 64, 1),
    (1, 1, 16, 1, 2048, 0),
    (1, 2, 8, 3, 100, 1),
    (4, 1, 32, 7, 16384, 0),
    (2, 2, 1, 64, 1 << 24, 1),
]


@pytest.fixture(autouse=True)
def _reset():
    api.tune_reset()
    yield
    api.tune_reset()


def _pin(op, tensors, shapes, counter, sched, params=None, bases=None):
    v, c, b, r, p, o = sched
    api.schedule_set(op, tensors, shapes=shapes, counter=counter, bases=bases, params=params,
                     vec_max=v, cache_policy=c, blocks_per_cu=b, box_rows_max=r, unit_elems=p,
                     unit_order=o)
    plan = api.describe(op, shapes, counter=counter, ptrs=[t.data_ptr() for t in tensors],
                        bases=bases, params=params)
    assert plan["cache_policy"] == c
    assert plan["unit_order"] == o
    assert plan["vec"] <= v
    return plan


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("d", [2, 4, 7])
def test_copy_pad_embed_every_schedule(sched, d):
    src_s, dst_s = inputs.cfg2_pad_shapes(d, log2_target=15)
    announce("copy schedule", d, src_s, dst_s, sched)
    src = inputs.uniform(2, src_s, 110, d)
    want = np.zeros(dst_s, dtype=np.float32)
    oracle.copy(src_s, want.reshape(-1), dst_s, src.reshape(-1), src_s)
    g = torch.zeros(dst_s, dtype=torch.float32, device="cuda")
    s = dev(src)
    _pin(L.OP_COPY, [g, s], [dst_s, src_s], src_s, sched, L.CopyParams(4))
    api.pad_embed_into(g, s)
    got = host(g)
    assert bits_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("sched", SCHEDULES)
@pytest.mark.parametrize("d", [3, 5, 8])
def test_mul_acc_every_schedule(sched, d):
    xs, ys, zs = inputs.cfg2_inter_shapes(d, log2_target=15)
    announce("mul_acc schedule", d, xs, ys, zs, sched)
    x = inputs.uniform(2, xs, 120, d)
    y = inputs.uniform(2, ys, 121, d)
    z = inputs.uniform(2, zs, 122, d)
    want = x.copy()
    oracle.mul_acc(xs, want.reshape(-1), xs, y.reshape(-1), ys, z.reshape(-1), zs)
    gx, gy, gz = dev(x), dev(y), dev(z)
    _pin(L.OP_MUL_ACC, [gx, gy, gz], [xs, ys, zs], None, sched)
    api.mul_acc_(gx, gy, gz)
    got = host(gx)
    assert bits_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("sched", SCHEDULES)
def test_embed_fill_every_schedule(sched):
    sx, dst_s = (13, 7, 30), (20, 9, 45)
    announce("embed_fill schedule", sx, dst_s, sched)
    x = inputs.rng(4, 130).standard_normal(sx).astype(np.float32)
    want = np.full(dst_s, 9.0, dtype=np.float32)
    oracle.embed_fill(dst_s, want.reshape(-1), dst_s, x.reshape(-1), sx)
    g = torch.full(dst_s, 9.0, dtype=torch.float32, device="cuda")
    gxx = dev(x)
    _pin(L.OP_EMBED_FILL, [g, gxx], [dst_s, sx], None, sched, L.CopyParams(4))
    api.embed_fill_(g, gxx)
    got = host(g)
    assert bits_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("sched", SCHEDULES)
def test_mul_and_adjoint_every_schedule(sched):
    so, sa, sb = (28, 30, 32, 26, 32), (32,) * 5, (28, 30, 32, 26, 32)
    announce("mul schedule", sched)
    a = inputs.rng(5, 140).standard_normal(sa).astype(np.float32)
    b = inputs.rng(5, 141).standard_normal(sb).astype(np.float32)
    want = np.zeros(so, dtype=np.float32)
    oracle.mul(so, want.reshape(-1), so, a.reshape(-1), sa, b.reshape(-1), sb)
    out = torch.empty(so, dtype=torch.float32, device="cuda")
    ga, gb = dev(a), dev(b)
    _pin(L.OP_MUL, [out, ga, gb], [so, sa, sb], so, sched)
    api.mul_into(out, ga, gb, counter=so)
    got = host(out)
    assert bits_equal(got, want), first_mismatch(got, want)

    announce("mul_adj schedule", sched)
    g = inputs.rng(5, 142).standard_normal(so).astype(np.float32)
    wa = np.full(sa, 5.0, dtype=np.float32)
    wb = np.full(sb, 5.0, dtype=np.float32)
    oracle.mul_adj(wa.reshape(-1), sa, wb.reshape(-1), sb, g.reshape(-1), so, a.reshape(-1),
                   b.reshape(-1))
    gg = dev(g)
    oa = torch.empty(sa, dtype=torch.float32, device="cuda")
    ob = torch.empty(sb, dtype=torch.float32, device="cuda")
    _pin(L.OP_MUL_ADJ, [oa, ob, gg, ga, gb], [sa, sb, so, sa, sb], None, sched)
    api.apply(L.OP_MUL_ADJ, [oa, ob, gg, ga, gb], [sa, sb, so, sa, sb], None, None, None,
              what="mul_adj")
    assert bits_equal(host(oa), wa), first_mismatch(host(oa), wa)
    assert bits_equal(host(ob), wb), first_mismatch(host(ob), wb)


def test_schedule_set_rejects_bad_knobs_and_row_kernels():
    announce("schedule_set errors")
    x = torch.zeros((8, 8), device="cuda")
    for bad in [(3, 1, 4, 1024, 8192, 0), (4, 3, 4, 1024, 8192, 0), (4, 1, 0, 1024, 8192, 0),
                (4, 1, 4, 2048, 8192, 0), (4, 1, 4, 1024, 32, 0), (4, 1, 4, 1024, 8192, 2)]:
        with pytest.raises(L.TriotError) as e:
            _pin(L.OP_COPY, [x, x.clone()], [(8, 8), (8, 8)], None, bad, L.CopyParams(4))
        assert e.value.status == L.E_INVALID
    with pytest.raises(L.TriotError) as e:
        api.schedule_set(L.OP_MOMENTS, [x], params=L.MomentsParams(0, 0))
    assert e.value.status == L.E_UNSUPPORTED


# Vector lanes over rows that start at any word: the inner extent is a
# multiple of 4 but outer strides and bases are not.
VEC_CASES = [
    # (counter, dst shape, src shape, dst base, src base)
    ((33, 64), (40, 67), (33, 64), 0, 0),
    ((9, 7, 12), (10, 9, 15), (11, 8, 17), 3, 5),
    ((5, 1000), (6, 1001), (7, 1003), 1001 + 1, 2 * 1003 + 3),
]


@pytest.mark.parametrize("case", range(len(VEC_CASES)))
@pytest.mark.parametrize("cp", [0, 1, 2])
def test_vector_lanes_on_word_aligned_rows(case, cp):
    counter, ds, ss, db, sb = VEC_CASES[case]
    announce("vec4 unaligned rows", counter, ds, ss, db, sb, cp)
    rng = np.random.default_rng(150 + case)
    src = rng.standard_normal(ss).astype(np.float32)
    dst = np.full(ds, 7.0, dtype=np.float32)
    want = dst.copy()
    oracle.copy(counter, want.reshape(-1), ds, src.reshape(-1), ss, db, sb)
    g, gs = dev(dst), dev(src)
    plan = _pin(L.OP_COPY, [g, gs], [ds, ss], counter, (4, cp, 4, 1024, 8192, 0),
                L.CopyParams(4), bases=[db, sb])
    assert plan["vec"] == 4
    api.copy_(g, gs, counter=counter, dst_base=db, src_base=sb)
    got = host(g)
    assert bits_equal(got, want), first_mismatch(got, want)
    # x += y * z with the same misaligned row starts
    announce("vec4 unaligned mul_acc", counter, cp)
    y = rng.standard_normal(ss).astype(np.float32)
    z = rng.standard_normal(ds).astype(np.float32)
    x = rng.standard_normal(counter).astype(np.float32)
    want = x.copy()
    oracle.mul_acc(counter, want.reshape(-1), counter, y.reshape(-1), ss, z.reshape(-1), ds)
    gx, gy, gz = dev(x), dev(y), dev(z)
    plan = _pin(L.OP_MUL_ACC, [gx, gy, gz], [counter, ss, ds], None, (4, cp, 4, 1024, 8192, 1))
    assert plan["vec"] == 4
    api.mul_acc_(gx, gy, gz)
    got = host(gx)
    assert bits_equal(got, want), first_mismatch(got, want)


def test_sequence_tuning_pins_schedules_and_keeps_results():
    """tune_sequence pins a schedule per problem of a sequence; the
    sequence still gives the oracle's bits afterwards."""
    from paper_1608_00099_amd import tune
    announce("sequence tuning")
    src_s, dst_s = (37, 41, 39), (40, 45, 44)
    xs, ys, zs = (33, 20, 39), (35, 21, 40), (33, 22, 41)
    rng = np.random.default_rng(160)
    src = rng.standard_normal(src_s).astype(np.float32)
    x = rng.standard_normal(xs).astype(np.float32)
    y = rng.standard_normal(ys).astype(np.float32)
    z = rng.standard_normal(zs).astype(np.float32)
    g, gs = torch.zeros(dst_s, device="cuda"), dev(src)
    gx, gy, gz = dev(x), dev(y), dev(z)
    runs = [0]

    def step_copy():
        api.pad_embed_into(g, gs)

    def step_mul_acc():
        runs[0] += 1
        api.mul_acc_(gx, gy, gz)

    problems = [dict(op=L.OP_COPY, tensors=[g, gs], counter=src_s, params=L.CopyParams(4)),
                dict(op=L.OP_MUL_ACC, tensors=[gx, gy, gz])]
    scheds = tune.tune_sequence(problems, [step_copy, step_mul_acc], steps=3,
                                knobs=(("vec_max", (4, 1)), ("cache_policy", (0, 1))))
    assert len(scheds) == 2
    for p, s in zip(problems, scheds):
        assert api.schedule_get(p["op"], p["tensors"], counter=p.get("counter"),
                                params=p.get("params")) == s
    want = np.zeros(dst_s, dtype=np.float32)
    oracle.copy(src_s, want.reshape(-1), dst_s, src.reshape(-1), src_s)
    assert bits_equal(host(g), want), first_mismatch(host(g), want)
    # x was updated `runs` times: replay that on the oracle
    gx.copy_(dev(x))
    api.mul_acc_(gx, gy, gz)
    want = x.copy()
    oracle.mul_acc(xs, want.reshape(-1), xs, y.reshape(-1), ys, z.reshape(-1), zs)
    assert bits_equal(host(gx), want), first_mismatch(host(gx), want)
    assert runs[0] > 1


def test_schedule_get_reports_defaults_and_pins():
    announce("schedule_get")
    x = torch.zeros((8, 40), device="cuda")
    y = torch.zeros((8, 40), device="cuda")
    z = torch.zeros((8, 40), device="cuda")
    s = api.schedule_get(L.OP_MUL_ACC, [x, y, z])
    assert s == {"vec_max": 4, "cache_policy": 1, "blocks_per_cu": 4, "box_rows_max": 1024,
                 "unit_elems": 8192, "unit_order": 0}
    _pin(L.OP_MUL_ACC, [x, y, z], [(8, 40)] * 3, None, (2, 2, 8, 16, 1024, 1))
    s = api.schedule_get(L.OP_MUL_ACC, [x, y, z])
    assert s == {"vec_max": 2, "cache_policy": 2, "blocks_per_cu": 8, "box_rows_max": 16,
                 "unit_elems": 1024, "unit_order": 1}
    with pytest.raises(L.TriotError) as e:
        api.schedule_get(L.OP_MOMENTS, [x], params=L.MomentsParams(0, 0))
    assert e.value.status == L.E_UNSUPPORTED


def test_rank_alone_and_seeded_sequence_tuning():
    """rank_alone times a grid for one problem and restores its schedule;
    tune_sequence seeded with candidates pins one schedule per problem and
    the results keep the oracle's bits."""
    from paper_1608_00099_amd import tune
    announce("rank alone")
    xs, ys, zs = (40, 37), (41, 39), (40, 38)
    rng = np.random.default_rng(170)
    x = rng.standard_normal(xs).astype(np.float32)
    y = rng.standard_normal(ys).astype(np.float32)
    z = rng.standard_normal(zs).astype(np.float32)
    gx, gy, gz = dev(x), dev(y), dev(z)
    prob = dict(op=L.OP_MUL_ACC, tensors=[gx, gy, gz])
    before = api.schedule_get(L.OP_MUL_ACC, [gx, gy, gz])
    grid = dict(vec_max=(4, 1), cache_policy=(0, 1), blocks_per_cu=(1, 4))
    ranked = tune.rank_alone(prob, lambda: api.mul_acc_(gx, gy, gz), grid=grid, reps=3)
    assert len(ranked) == 8
    assert [t for t, _ in ranked] == sorted(t for t, _ in ranked)
    assert api.schedule_get(L.OP_MUL_ACC, [gx, gy, gz]) == before
    scheds = tune.tune_sequence([prob], [lambda: api.mul_acc_(gx, gy, gz)], steps=3,
                                knobs=(), passes=1, candidates=[[s for _, s in ranked[:3]]])
    assert scheds[0] in [before] + [s for _, s in ranked[:3]]
    gx.copy_(dev(x))
    api.mul_acc_(gx, gy, gz)
    want = x.copy()
    oracle.mul_acc(xs, want.reshape(-1), xs, y.reshape(-1), ys, z.reshape(-1), zs)
    assert bits_equal(host(gx), want), first_mismatch(host(gx), want)
