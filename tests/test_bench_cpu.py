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
