"""Host-side checks of bench.py: the --gpus contract and the pinned launch
schedules of the sweep."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_pinned_schedules_cover_every_sweep_launch_with_valid_knobs():
    with open(bench.SCHEDULES) as f:
        saved = json.load(f)
    names = ["%s d=%d" % (k, d) for d in range(2, 9) for k in ("copy", "mul_acc")]
    assert sorted(saved) == sorted(names)
    for name, s in saved.items():
        assert set(s) == {"vec_max", "cache_policy", "blocks_per_cu", "box_rows_max",
                          "unit_elems", "unit_order"}, name
        assert s["vec_max"] in (1, 2, 4)
        assert s["cache_policy"] in (0, 1, 2)
        assert 1 <= s["blocks_per_cu"] <= 32
        assert 1 <= s["box_rows_max"] <= 1024
        assert 64 <= s["unit_elems"] <= 1 << 24
        assert s["unit_order"] in (0, 1)


def _points(counter, shape, base):
    import itertools
    out = []
    for t in itertools.product(*[range(c) for c in counter]):
        off, st = 0, 1
        for i in range(len(counter) - 1, -1, -1):
            off += t[i] * st
            st *= shape[i]
        out.append(base + off)
    return out


def test_cpu_timing_windows_cover_the_counter_once():
    """The threaded oracle timing splits the counter into windows of its
    leading axes: together they visit every point of every operand once."""
    cases = [((3, 4, 5), [(4, 6, 7), (3, 4, 5)], 8),
             ((2, 3, 4, 5), [(3, 3, 6, 5), (2, 3, 4, 5)], 16),
             ((7,), [(9,)], 4),
             ((2, 2, 2, 2, 3), [(3, 3, 3, 3, 3)], 64)]
    for counter, shapes, pieces in cases:
        wins = bench._slabs(counter, shapes, [0] * len(shapes), pieces)
        assert len(wins) >= min(pieces, len(_points(counter[:-1] or (1,), counter[:-1] or (1,), 0)))
        for k, shape in enumerate(shapes):
            got = [p for sub, bs in wins for p in _points(sub, shape, bs[k])]
            assert sorted(got) == sorted(_points(counter, shape, 0))


def test_cpu_baseline_runs_small():
    r = bench.cpu_baseline(12, 3)
    assert r["single"][0] > 0 and r["threaded"][0] > 0
    assert r["threaded"][1] <= r["threaded"][0] <= r["threaded"][2]
