"""Tuning the schedules of a sequence of co-iterations where they run.

triot_autotune times one problem alone, after a cache flush.  In a
pipeline each launch instead runs after other kernels over other buffers,
and the write-backs of lines it leaves dirty are paid by the launch after
it, so the fastest schedule of a problem alone is not always the fastest
in its sequence.  tune_sequence refines the schedules of a list of
problems by coordinate descent on their in-sequence times: for each
problem, each value of each knob is pinned (triot_schedule_set) and the
whole sequence is run a few times with HIP events between the launches;
the objective of problem i is the median time of launch i plus launch
i + 1.  rank_alone times a whole grid of schedules for one problem alone
(cold), whose fastest few seed that search.  Results do not depend on the
schedule (only the speed does).
"""
from __future__ import annotations

import itertools

import torch

from . import api

KNOBS = (("vec_max", (4, 2, 1)), ("cache_policy", (0, 1, 2)), ("blocks_per_cu", (1, 2, 4, 8)))

# The full grid ranked alone (cold) before the in-sequence refinement.
GRID = dict(vec_max=(4, 2, 1), cache_policy=(0, 1, 2), blocks_per_cu=(1, 2, 4, 8, 16),
            unit_order=(0, 1), box_rows_max=(64, 1024),
            unit_elems=(2048, 4096, 8192, 16384, 32768))


def _key(p):
    return dict(shapes=p.get("shapes"), counter=p.get("counter"), bases=p.get("bases"),
                params=p.get("params"))


def rank_alone(problem, launch, grid=GRID, reps=5, flush=None):
    """Every schedule of `grid` for one problem, timed alone with HIP events
    (median of `reps`), each run after a write over `flush` (a device
    tensor larger than the memory-side cache) when given.  Returns
    [(ms, schedule)] fastest first and pins the schedule the problem had
    before."""
    saved = api.schedule_get(problem["op"], problem["tensors"], **_key(problem))
    names = list(grid)
    s = torch.cuda.current_stream()
    out = []
    for values in itertools.product(*(grid[n] for n in names)):
        sched = dict(saved)
        sched.update(zip(names, values))
        api.schedule_set(problem["op"], problem["tensors"], **_key(problem), **sched)
        launch()
        ms = []
        for _ in range(reps):
            if flush is not None:
                flush.fill_(0.0)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(s)
            launch()
            b.record(s)
            b.synchronize()
            ms.append(a.elapsed_time(b))
        ms.sort()
        out.append((ms[len(ms) // 2], sched))
    api.schedule_set(problem["op"], problem["tensors"], **_key(problem), **saved)
    out.sort(key=lambda t: t[0])
    return out


def _times(launches, steps):
    """Per-launch in-sequence times (ms), one list per step."""
    s = torch.cuda.current_stream()
    n = len(launches)
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(n + 1)] for _ in range(steps)]
    for f in launches:      # one untimed pass
        f()
    for k in range(steps):
        for i, f in enumerate(launches):
            ev[k][i].record(s)
            f()
        ev[k][n].record(s)
    torch.cuda.synchronize()
    return [[ev[k][i].elapsed_time(ev[k][i + 1]) for i in range(n)] for k in range(steps)]


def _objective(launches, i, steps):
    """Median over steps of launch i plus the launch after it (the sequence
    repeats: the last launch is followed by the first)."""
    n = len(launches)
    v = sorted(t[i] + (t[(i + 1) % n] if n > 1 else 0.0) for t in _times(launches, steps))
    return v[len(v) // 2]


def tune_sequence(problems, launches, steps=7, knobs=KNOBS, passes=2, min_gain=0.005, log=None,
                  candidates=None):
    """problems[i]: dict(op=, tensors=, shapes=, counter=, bases=, params=)
    describing what launches[i] (a callable) runs.  Pins, for every
    problem, the best schedule found and returns them (a list of dicts in
    schedule_set's keywords).  `candidates[i]` (optional): whole schedules
    tried for problem i before the knob-by-knob descent (e.g. the fastest
    few of rank_alone).  `passes` sweeps over the problems (later problems'
    schedules change the earlier ones' surroundings).  A candidate replaces
    the current schedule only when it cuts the objective by more than
    `min_gain` (relative)."""
    key = _key
    scheds = [api.schedule_get(p["op"], p["tensors"], **key(p)) for p in problems]
    for ps in range(passes):
        for i, p in enumerate(problems):
            best = dict(scheds[i])
            api.schedule_set(p["op"], p["tensors"], **key(p), **best)
            best_t = _objective(launches, i, steps)
            if ps == 0 and candidates is not None:
                for cand in candidates[i]:
                    if cand == best:
                        continue
                    api.schedule_set(p["op"], p["tensors"], **key(p), **cand)
                    t = _objective(launches, i, steps)
                    if t < best_t * (1.0 - min_gain):
                        best, best_t = dict(cand), t
                api.schedule_set(p["op"], p["tensors"], **key(p), **best)
            for name, values in knobs:
                for v in values:
                    if v == best[name]:
                        continue
                    cand = dict(best)
                    cand[name] = v
                    api.schedule_set(p["op"], p["tensors"], **key(p), **cand)
                    t = _objective(launches, i, steps)
                    if t < best_t * (1.0 - min_gain):
                        best, best_t = cand, t
                api.schedule_set(p["op"], p["tensors"], **key(p), **best)
            scheds[i] = best
            if log:
                log("sequence tuning pass %d: problem %d -> %s (%.1f us with the next launch)"
                    % (ps, i, best, best_t * 1e3))
    return scheds
