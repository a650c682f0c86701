"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every symbol include/triot.h declares, validation returns the
documented codes, the magic-division constants are exact, and the planner
drops and merges axes as described."""
import json
import os
import re

import numpy as np
import pytest

from paper_1608_00099_amd import _lib as L
from paper_1608_00099_amd import api

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "triot.h")

# Fake, non-overlapping device addresses: planning never dereferences them.
P0, P1, P2, P3, P4 = [(k + 1) << 40 for k in range(5)]


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(triot_[a-z_]+)\s*\(", text)))


def test_header_declares_and_library_exports_every_entry_point():
    names = declared_functions()
    assert "triot_apply" in names and "triot_apply_batched" in names
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n), "libtriot.so does not export %s" % n
    assert set(names) == set(L.EXPORTS)


def test_status_strings():
    for s in range(9):
        assert L.status_string(s)
    assert L.status_string(0) == "ok"


def _apply(op, shapes, counter=None, ptrs=None, bases=None, params=None, out=0, ws=0, wsb=0):
    d = len(shapes[0]) if shapes else 0
    ptrs = ptrs if ptrs is not None else [P0, P1, P2, P3, P4][: len(shapes)]
    return L.triot_apply(op, len(shapes), d, shapes, counter, ptrs, bases, params, out, ws, wsb, 0)


def test_validation_codes():
    # wrong operand count / op
    assert _apply(L.OP_COPY, [(4,), (4,), (4,)]) == L.E_INVALID
    assert L.triot_apply(99, 2, 1, [(4,), (4,)], None, [P0, P1], None, None, 0, 0, 0, 0) == L.E_INVALID
    # dimension
    assert L.triot_apply(L.OP_COPY, 2, 33, [(1,) * 33, (1,) * 33], None, [P0, P1], None, None,
                         0, 0, 0, 0) == L.E_DIM
    assert L.triot_apply(L.OP_COPY, 2, -1, [], None, [P0, P1], None, None, 0, 0, 0, 0) == L.E_DIM
    # counter beyond an operand (the paper's bounds check)
    assert _apply(L.OP_COPY, [(4, 4), (3, 5)], counter=(4, 4)) == L.E_BOUNDS
    # window beyond the parent
    assert _apply(L.OP_COPY, [(6, 6), (6, 6)], counter=(3, 3), bases=[4 * 6, 0]) == L.E_BOUNDS
    assert _apply(L.OP_COPY, [(6, 6), (6, 6)], counter=(3, 3), bases=[36, 0]) == L.E_BOUNDS
    # null pointer with work
    assert _apply(L.OP_COPY, [(4,), (4,)], ptrs=[P0, 0]) == L.E_INVALID
    # null pointers without work are fine: extent 0 is a no-op
    assert _apply(L.OP_COPY, [(4, 0), (4, 0)], ptrs=[0, 0]) == L.OK
    # partial overlap of the output with an input
    assert _apply(L.OP_COPY, [(8,), (8,)], counter=(8,), ptrs=[P0, P0 + 8]) == L.E_ALIAS
    assert _apply(L.OP_MUL_ACC, [(8,), (8,), (8,)], ptrs=[P0, P0 + 4, P2]) == L.E_ALIAS
    # the exact same view as input of an element-wise op is allowed
    st, _ = L.triot_plan_describe(L.OP_MUL_ACC, 3, 1, [(8,), (8,), (8,)], None, [P0, P1, P0])
    assert st == L.OK
    # overflow of an int64 size
    big = (1 << 31, 1 << 31, 1 << 3)
    assert _apply(L.OP_COPY, [big, big], counter=(1, 1, 1)) == L.E_OVERFLOW
    # bad params
    assert _apply(L.OP_COPY, [(4,), (4,)], params=L.CopyParams(3)) == L.E_INVALID
    assert _apply(L.OP_MOMENTS_ADJ, [(4,)]) == L.E_INVALID
    # moments need a workspace and an output
    assert _apply(L.OP_MOMENTS, [(4, 4)], out=P3) == L.E_WORKSPACE
    assert _apply(L.OP_MOMENTS, [(4, 4)], out=0, ws=P2, wsb=1 << 20) == L.E_INVALID
    # covariance beyond 8 axes is outside this build's limits
    shp = (2,) * 9
    st = _apply(L.OP_MOMENTS, [shp], out=P3, ws=P2, wsb=1 << 30,
                params=L.MomentsParams(L.MOMENTS_FIRST | L.MOMENTS_COV, None))
    assert st == L.E_UNSUPPORTED


def _magic_div(n, m, s):
    h = (n * m) >> 32
    return (h + ((n - h) >> 1)) >> s


def test_magic_division_exact_for_all_small_divisors():
    """Every divisor 2..2^16 against boundary numerators and random samples
    (Granlund & Montgomery's round-up method must equal floor division)."""
    rng = np.random.default_rng(0)
    top = (1 << 32) - 1
    cs = np.arange(2, (1 << 16) + 1, dtype=np.uint64)
    ms = np.empty_like(cs)
    ss = np.empty_like(cs)
    for i, c in enumerate(cs):
        st, m, s = L.triot_divmod_magic(int(c))
        assert st == L.OK
        ms[i], ss[i] = m, s
    for k in [0, 1, 2, 3]:
        # numerators: 0, c-1, c, k*c - 1 near the top, 2^32 - 1, random
        nums = [np.zeros_like(cs), cs - 1, cs, (top // cs) * cs - 1, (top // cs) * cs,
                np.full_like(cs, top), rng.integers(0, top, size=cs.size, dtype=np.uint64)][k::4]
        for n in nums:
            h = (n * ms) >> np.uint64(32)
            q = (h + ((n - h) >> np.uint64(1))) >> ss
            assert np.array_equal(q, n // cs)


def test_magic_division_large_divisors():
    rng = np.random.default_rng(1)
    top = (1 << 32) - 1
    for c in list(rng.integers(1 << 16, top, size=2000)) + [top, top - 1, (1 << 31) + 1, 1 << 31]:
        c = int(c)
        st, m, s = L.triot_divmod_magic(c)
        assert st == L.OK
        for n in [0, c - 1, c, min(2 * c - 1, top), top, int(rng.integers(0, top))]:
            assert _magic_div(n, m, s) == n // c
    assert L.triot_divmod_magic(1)[0] == L.E_INVALID
    assert L.triot_divmod_magic(0)[0] == L.E_INVALID


def test_plan_drops_extent_one_and_merges_full_axes():
    # cfg1: (48,40,36) into (64,64,64): nothing merges, inner extent 36
    p = api.describe(L.OP_COPY, [(64, 64, 64), (48, 40, 36)], counter=(48, 40, 36))
    assert p["dims"] == 3 and p["extents"] == [48, 40, 36]
    assert p["vec"] == 4                      # 36 and the strides are multiples of 4
    # a full operand pair collapses to one flat axis
    p = api.describe(L.OP_MUL_ACC, [(16,) * 6] * 3)
    assert p["dims"] == 1 and p["extents"] == [16 ** 6]
    # extent-1 counter axes are dropped
    p = api.describe(L.OP_COPY, [(5, 7, 9), (5, 7, 9)], counter=(5, 1, 9))
    assert p["dims"] == 2 and p["extents"] == [5, 9]
    # the differentiable workload's product: (28,30,32,26,32) in 32^5
    p = api.describe(L.OP_MUL, [(28, 30, 32, 26, 32), (32,) * 5, (28, 30, 32, 26, 32)])
    assert p["extents"] == [28, 960, 832]
    # 8-byte copies move two words per element
    p = api.describe(L.OP_COPY, [(10, 10), (6, 7)], counter=(6, 7), params=L.CopyParams(8))
    assert p["extents"] == [6, 14]
    # scalars
    p = api.describe(L.OP_COPY, [(), ()])
    assert p["dims"] == 1 and p["extents"] == [1]


def test_plan_ragged_rows():
    # an inner extent that is not a multiple of 4: 4-word lanes, each row's
    # last vector holding 39 % 4 = 3 new words
    p = api.describe(L.OP_MUL_ACC, [(57, 59, 37, 15, 39), (62, 59, 44, 22, 51),
                                    (59, 64, 40, 19, 41)])
    assert p["vec"] == 4 and p["row_tail"] == 3 and p["extents"][-1] == 39
    p = api.describe(L.OP_COPY, [(10, 11), (6, 9)], counter=(6, 9))
    assert p["vec"] == 4 and p["row_tail"] == 1 and p["extents"] == [6, 9]
    # 3 words: 2-word lanes, the last one moved back by a word
    p = api.describe(L.OP_MUL, [(7, 3), (7, 3), (7, 5)])
    assert p["vec"] == 2 and p["row_tail"] == 1
    # whole vectors report no tail
    p = api.describe(L.OP_MUL_ACC, [(5, 40), (5, 44), (5, 48)])
    assert p["vec"] == 4 and p["row_tail"] == 0
    # EMBED_FILL: ragged destination rows and a source bound at any word
    p = api.describe(L.OP_EMBED_FILL, [(9, 11), (7, 9)], params=L.CopyParams(4))
    assert p["vec"] == 4 and p["row_tail"] == 3
    # the adjoint product (window predicates on several operands) keeps
    # 1-word lanes on ragged rows, as does a row of at most one vector
    p = api.describe(L.OP_MUL_ADJ, [(6, 9), (6, 7), (6, 7), (6, 9), (6, 7)])
    assert p["vec"] == 1 and p["row_tail"] == 0
    p = api.describe(L.OP_MUL_ACC, [(5, 2), (5, 3), (5, 3)])
    assert p["vec"] == 1 and p["row_tail"] == 0
    # one row of 4190211 elements: 1047553 vectors in 1024 units of 1024, so
    # the last unit holds only the ragged vector (its offsets are taken from
    # the vector before the unit, never from before the row)
    p = api.describe(L.OP_COPY, [(4190211,), (4190211,)], params=L.CopyParams(4))
    assert p["vec"] == 4 and p["row_tail"] == 3 and p["units"] == 1024 and p["box_rows"] == 1


def test_default_schedules_by_problem_size():
    """Without a pinned or tuned schedule: 4 workgroups per CU and
    contiguous unit ranges, or, for copies and products of at least 2^25
    counter points, 1 per CU and round-robin units (no device work)."""
    def get(shapes, op=L.OP_MUL_ACC, params=None):
        ptrs = [(k + 1) << 40 for k in range(len(shapes))]
        st, sch = L.triot_schedule_get(op, len(shapes), len(shapes[0]), shapes, None,
                                       ptrs, None, params)
        assert st == L.OK
        return (sch.vec_max, sch.cache_policy, sch.blocks_per_cu, sch.box_rows_max,
                sch.unit_elems, sch.unit_order)
    api.tune_reset()
    assert get([(8, 40)] * 3) == (4, 1, 4, 1024, 8192, 0)
    assert get([(1 << 12, (1 << 13) - 1)] * 3) == (4, 1, 4, 1024, 8192, 0)
    assert get([(1 << 12, 1 << 13)] * 3) == (4, 1, 1, 1024, 8192, 1)
    # the counter, not the operands, decides: a small window of large tensors
    assert get([(1 << 12, 8), (1 << 13, 1 << 13), (1 << 13, 1 << 13)]) == (4, 1, 4, 1024, 8192, 0)
    big = [(1 << 12, 1 << 13)] * 2
    assert get(big, L.OP_COPY, L.CopyParams(4)) == (4, 1, 1, 1024, 8192, 1)
    # a large EMBED_FILL keeps 4 workgroups per CU and contiguous ranges
    assert get(big, L.OP_EMBED_FILL, L.CopyParams(4)) == (4, 1, 4, 1024, 8192, 0)


def test_plan_box_split_limits():
    # very short rows: the box tabulates several low axes (bounded table)
    p = api.describe(L.OP_COPY, [(9, 5, 13, 21, 14, 6, 3, 25)] * 1 + [(10, 6, 14, 22, 15, 7, 4, 26)],
                     counter=(9, 5, 13, 21, 14, 6, 3, 25))
    assert p["box_rows"] <= 1024
    assert p["low_axes"] >= 1
    assert p["units"] >= p["blocks"]
    # one very long row: a single-row box split into units
    p = api.describe(L.OP_COPY, [(1 << 24,), (1 << 24,)])
    assert p["box_rows"] == 1 and p["units"] > 1


def test_segment_plan_for_moments():
    p = api.describe(L.OP_MOMENTS, [(16,) * 6])
    assert p["kernel"] == 1 and p["dims"] == 6 and p["extents"] == [16] * 6
    p = api.describe(L.OP_MOMENTS, [(3, 1, 5)])
    assert p["dims"] == 2 and p["extents"] == [3, 5]


def test_workspace_size():
    assert L.triot_workspace_size(L.OP_COPY, 2, 1, [(4,), (4,)]) == 0
    n = L.triot_workspace_size(L.OP_MOMENTS, 1, 6, [(16,) * 6])
    assert n > 256


def _batched_status(op, items):
    st, h = L.triot_batch_create()
    assert st == L.OK
    try:
        return L.triot_apply_batched(op, items, None, h, 0)
    finally:
        L.triot_batch_destroy(h)


def test_batched_rejects_overlap_across_items():
    # Validation and the cross-item check run before any device call, so
    # with fake addresses a rejected batch returns E_ALIAS here (a batch
    # that passes would need a device and fails later with E_DEVICE).
    sh = [(4, 4), (4, 4)]
    n16 = 16 * 4   # bytes of one (4, 4) float32 tensor
    # item 1 writes into item 0's source
    items = [(2, 2, sh, None, [P0, P1], None), (2, 2, sh, None, [P1, P2], None)]
    assert _batched_status(L.OP_COPY, items) == L.E_ALIAS
    # two outputs overlap by one element
    items = [(2, 2, sh, None, [P0, P1], None), (2, 2, sh, None, [P0 + n16 - 4, P2], None)]
    assert _batched_status(L.OP_COPY, items) == L.E_ALIAS
    # an output inside another item's window read (bases make the window)
    items = [(2, 2, [(4, 4), (8, 8)], (4, 4), [P0, P1], [0, 4 * 8 + 4]),
             (2, 2, [(2, 2), (2, 2)], None, [P1 + (5 * 8 + 5) * 4, P2], None)]
    assert _batched_status(L.OP_EMBED_FILL, items) == L.E_ALIAS
    # x += y*z with another item's x as its y
    s3 = [(4, 4)] * 3
    items = [(2, 3, s3, None, [P0, P1, P2], None), (2, 3, s3, None, [P3, P0, P4], None)]
    assert _batched_status(L.OP_MUL_ACC, items) == L.E_ALIAS
    # the same view in and out within one item stays legal, and so do
    # inputs shared by several items and adjacent outputs: these pass the
    # checks and stop only at the device query
    ok = {L.E_DEVICE, L.OK}
    items = [(2, 3, s3, None, [P0, P0, P2], None), (2, 3, s3, None, [P3, P2, P2], None)]
    assert _batched_status(L.OP_MUL_ACC, items) in ok
    items = [(2, 2, sh, None, [P0, P2], None), (2, 2, sh, None, [P0 + n16, P2], None)]
    assert _batched_status(L.OP_COPY, items) in ok


def test_batched_overlap_check_many_items():
    # 512 items writing adjacent blocks and all reading one shared source:
    # accepted by the checks; moving one output back by one element makes
    # it overlap its neighbour.
    n = 512
    sh = [(8,), (8,)]
    items = [(1, 2, sh, None, [P0 + 32 * i, P1], None) for i in range(n)]
    assert _batched_status(L.OP_COPY, items) in {L.E_DEVICE, L.OK}
    items[300] = (1, 2, sh, None, [P0 + 32 * 300 - 4, P1], None)
    assert _batched_status(L.OP_COPY, items) == L.E_ALIAS


def test_tune_cache_file_skips_corrupt_lines(tmp_path):
    """TRIOT_TUNE_CACHE: well-formed entries are loaded; garbage, truncated
    lines and entries with out-of-range knobs are ignored (defaults stay).
    In a fresh process, since the file is read once per process."""
    import subprocess
    import sys
    cache = tmp_path / "tune.jsonl"
    script = tmp_path / "probe.py"
    script.write_text(r'''
import json, os, sys
sys.path.insert(0, %r)
from paper_1608_00099_amd import _lib as L

def key(shape):
    s = ":s%%d,%%d,b0,a0" %% shape
    return "op%%d:n3:e4:d2:c%%d,%%d," %% ((L.OP_MUL_ACC,) + shape) + s * 3

def get(shape):
    ptrs = [(k + 1) << 40 for k in range(3)]
    st, s = L.triot_schedule_get(L.OP_MUL_ACC, 3, 2, [shape] * 3, None, ptrs, None, None)
    assert st == L.OK
    return [s.vec_max, s.cache_policy, s.blocks_per_cu, s.box_rows_max, s.unit_elems, s.unit_order]

if sys.argv[1] == "keys":
    print(json.dumps([key((8, 40)), key((9, 40)), key((10, 40))]))
else:
    print(json.dumps([get((8, 40)), get((9, 40)), get((10, 40))]))
''' % ROOT)
    env = dict(os.environ)
    env.pop("TRIOT_TUNE_CACHE", None)
    keys = json.loads(subprocess.run([sys.executable, str(script), "keys"], env=env, check=True,
                                     capture_output=True, text=True).stdout)
    cache.write_text("\n".join([
        "not a cache line",
        '{"key": "%s", "vec": 2, "cache": 0, "bpc": 8, "order": 1, "rb": 64, "pe": 2048}' % keys[0],
        '{"key": "%s", "vec": 3, "cache": 0, "bpc": 8, "order": 1, "rb": 64, "pe": 2048}' % keys[1],
        '{"key": "%s", "vec": 4, "cache": 1' % keys[2],
        "",
    ]) + "\n")
    env["TRIOT_TUNE_CACHE"] = str(cache)
    got = json.loads(subprocess.run([sys.executable, str(script), "get"], env=env, check=True,
                                    capture_output=True, text=True).stdout)
    default = [4, 1, 4, 1024, 8192, 0]
    assert got[0] == [2, 0, 8, 64, 2048, 1]
    assert got[1] == default and got[2] == default
