#!/usr/bin/env python3
"""Benchmark of the co-iteration hot path on one MI355X.

One step = the run-time-dimension sweep d = 2..8 (the workload the headline
metric is quoted on): for every d, a zero-pad embedding of a ~2^26-element
float32 tensor into a shape enlarged by 1..16 per axis (COPY over the source
shape into a pre-zeroed destination) and x[t] += y[t]*z[t] over the
intersection of three shapes (MUL_ACC).  All tensors are resident in HBM
before timing.  `value` is the effective HBM bandwidth of the whole step:
algorithmic bytes (8 B per copied point, 16 B per x += y*z point) divided by
the step time.

Also reported on the same line: the roofline of the dominant kernel (HIP
events around its launches), the CPU oracle on a bounded sample of the same
workload, and per-configuration figures for the other parts of the hot path
(moments, batched padding for FFT convolution, the differentiable pipeline,
the small pad-embed) next to a plain device-copy ceiling.

The sweep's launch schedules are pinned from a JSON file written by an
earlier `--retune --save-schedules` run on an MI355X (a grid of schedules
ranked alone for every launch, then the in-sequence refinement of tune.py),
so that
every run and its profiles launch the same kernels; `--retune` tunes afresh.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]
                       [--retune] [--save-schedules FILE] [--schedules FILE] [--no-tune]
"""
import argparse
import gc
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# The sweep's launch schedules as tuned on an MI355X (bench.py --retune
# --save-schedules): pinned by default so that every run, and the profiles
# of it, launch the same kernels.
SCHEDULES = os.path.join(ROOT, "paper_1608_00099_amd", "tuned", "sweep_d2-8_mi355x.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def prod(s):
    p = 1
    for v in s:
        p *= int(v)
    return p


def kernel_source_hash():
    from paper_1608_00099_amd.profiling import kernel_source_hash as h
    return h()


# ---------------------------------------------------------------------------
# GPU workload
# ---------------------------------------------------------------------------

class Sweep:
    """The d = 2..8 sweep, resident on the device."""

    def __init__(self, dev, log2_target=26):
        import torch
        from paper_1608_00099_amd import inputs
        self.items = []
        seed = 1000
        for d in range(2, 9):
            src_s, dst_s = inputs.cfg2_pad_shapes(d, log2_target)
            xs, ys, zs = inputs.cfg2_inter_shapes(d, log2_target)
            src = inputs.uniform_torch(src_s, seed + 10 * d + 0, dev)
            dst = torch.zeros(dst_s, dtype=torch.float32, device=dev)
            x = inputs.uniform_torch(xs, seed + 10 * d + 1, dev)
            y = inputs.uniform_torch(ys, seed + 10 * d + 2, dev)
            z = inputs.uniform_torch(zs, seed + 10 * d + 3, dev)
            self.items.append(dict(d=d, src=src, dst=dst, x=x, y=y, z=z, src_s=src_s, dst_s=dst_s,
                                   xs=xs, ys=ys, zs=zs))
        torch.cuda.synchronize()

    def launches(self):
        """[(name, op, callable, algorithmic bytes)] of one step."""
        from paper_1608_00099_amd import api
        from paper_1608_00099_amd import _lib as L
        out = []
        for it in self.items:
            out.append(("copy d=%d" % it["d"], L.OP_COPY,
                        (lambda it=it: api.pad_embed_into(it["dst"], it["src"])),
                        8 * prod(it["src_s"]), it))
            out.append(("mul_acc d=%d" % it["d"], L.OP_MUL_ACC,
                        (lambda it=it: api.mul_acc_(it["x"], it["y"], it["z"])),
                        16 * prod(it["xs"]), it))
        return out


def plan_of(op, it):
    from paper_1608_00099_amd import api
    if op == 0:
        shapes, counter = [it["dst_s"], it["src_s"]], it["src_s"]
        ptrs = [it["dst"].data_ptr(), it["src"].data_ptr()]
    else:
        shapes, counter = [it["xs"], it["ys"], it["zs"]], None
        ptrs = [it["x"].data_ptr(), it["y"].data_ptr(), it["z"].data_ptr()]
    p = api.describe(op, shapes, counter=counter, ptrs=ptrs)
    return p, api.kernel_name(op, p)


def autotune_all(launches):
    """Let the library's autotuner pick each launch's schedule (it times the
    candidates with HIP events on these very buffers)."""
    from paper_1608_00099_amd import api
    for p in problems_of(launches):
        api.autotune(p["op"], p["tensors"], counter=p.get("counter"), params=p.get("params"))


def problems_of(launches):
    """The (op, operands) of every launch, as the schedule calls take them."""
    from paper_1608_00099_amd import _lib as L
    out = []
    for name, op, fn, nbytes, it in launches:
        if op == L.OP_COPY:
            out.append(dict(op=op, tensors=[it["dst"], it["src"]], counter=it["src_s"],
                            params=L.CopyParams(4)))
        else:
            out.append(dict(op=op, tensors=[it["x"], it["y"], it["z"]]))
    return out


def sequence_tune(launches, dev):
    """Rank a grid of schedules for every launch alone (cold), pin each
    launch's fastest, then refine in the sequence they run in, trying each
    launch's twelve fastest first (three passes; see tune.py)."""
    import torch
    from paper_1608_00099_amd import api, tune
    flush = torch.empty(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
    probs = problems_of(launches)
    cands = []
    for (name, op, fn, nbytes, it), p in zip(launches, probs):
        ranked = tune.rank_alone(p, fn, reps=3, flush=flush)
        api.schedule_set(p["op"], p["tensors"], counter=p.get("counter"), params=p.get("params"),
                         **ranked[0][1])
        cands.append([sched for _, sched in ranked[:12]])
        log("ranked %d schedules for %s alone: best %.1f us" % (len(ranked), name,
                                                                ranked[0][0] * 1e3))
    del flush
    tune.tune_sequence(probs, [x[2] for x in launches], log=log, candidates=cands, passes=3)


def save_schedules(launches, path):
    """Write the schedule every launch runs with (name -> schedule_set's
    keywords)."""
    from paper_1608_00099_amd import api
    out = {}
    for (name, *_), p in zip(launches, problems_of(launches)):
        out[name] = api.schedule_get(p["op"], p["tensors"], counter=p.get("counter"),
                                     params=p.get("params"))
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


def pin_schedules(launches, path):
    from paper_1608_00099_amd import api
    with open(path) as f:
        saved = json.load(f)
    missing = [x[0] for x in launches if x[0] not in saved]
    if missing:
        raise SystemExit("%s has no schedule for %s" % (path, missing))
    for (name, *_), p in zip(launches, problems_of(launches)):
        api.schedule_set(p["op"], p["tensors"], counter=p.get("counter"),
                         params=p.get("params"), **saved[name])


def tuned_summary(launches):
    out = {}
    for name, op, fn, nbytes, it in launches:
        p = plan_of(op, it)[0]
        out[name] = {"cache": p["cache_policy"], "blocks": p["blocks"], "vec": p["vec"],
                     "box_rows": p["box_rows"], "row_tail": p["row_tail"]}
    return out


def time_steps_plain(fns, steps, warmup):
    """Time exactly `steps` steps of the launch sequence `fns`, with HIP
    events only before the first and after the last launch (a marker
    between launches costs the device a few microseconds each).  Returns
    the step time (ms) and the host wall time per step (ms)."""
    import torch
    for _ in range(warmup):
        for f in fns:
            f()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    b.record(s)
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    try:
        t0 = time.perf_counter()
        a.record(s)
        for _ in range(steps):
            for f in fns:
                f()
        b.record(s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        gc.enable()
    return a.elapsed_time(b) / steps, wall / steps * 1e3


def time_steps(fns, steps, warmup):
    """Time exactly `steps` steps of the launch sequence `fns`.  HIP events
    recorded on the stream the kernels run on (the library enqueues on
    torch's current stream) bracket every launch inside the timed region, so
    each kernel's duration is the one it has in the real sequence (after a
    different kernel over other buffers, not after itself).  Returns the
    step time (ms, first to last event), the host wall time per step (ms)
    and the per-launch durations [launch][step] (ms)."""
    import torch
    for _ in range(warmup):
        for f in fns:
            f()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(fns) + 1)]
          for _ in range(steps)]
    # torch creates the HIP event at its first record: do that now, outside
    # the timed region (a creation stall would starve the device there).
    for row in ev:
        for e in row:
            e.record(s)
    torch.cuda.synchronize()
    # No garbage collection while the host enqueues the timed steps: a
    # collector pause would leave the device idle inside a timed launch.
    gc.collect()
    gc.disable()
    try:
        t0 = time.perf_counter()
        for k in range(steps):
            for i, f in enumerate(fns):
                ev[k][i].record(s)
                f()
            ev[k][len(fns)].record(s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    finally:
        gc.enable()
    total = ev[0][0].elapsed_time(ev[-1][len(fns)])
    per = [[ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(steps)] for i in range(len(fns))]
    return total / steps, wall / steps * 1e3, per


# ---------------------------------------------------------------------------
# CPU baseline: the oracle on a bounded sample of the same workload
# ---------------------------------------------------------------------------

def _slabs(counter, shapes, bases, pieces):
    """Split a counter into at least `pieces` windows along its leading
    axes: [(sub-counter, per-operand bases)], each a plain oracle call."""
    d = len(counter)
    k, n = 0, 1
    while k < d - 1 and n < pieces:
        n *= counter[k]
        k += 1
    out = []
    for f in range(n):
        t, r = [0] * k, f
        for i in range(k - 1, -1, -1):
            t[i] = r % counter[i]
            r //= counter[i]
        sub = tuple([1] * k + list(counter[k:])) if k else tuple(counter)
        bs = []
        for s_, b in zip(shapes, bases):
            stride, off = 1, 0
            for i in range(d - 1, -1, -1):
                if i < k:
                    off += t[i] * stride
                stride *= s_[i]
            bs.append(b + off)
        out.append((sub, bs))
    return out


def cpu_baseline(log2_target, threads):
    """The oracle on the sweep recipe: one single-threaded pass, then three
    passes with `threads` threads, each taking windows of the leading
    counter axes (plain oracle calls; ctypes releases the interpreter lock
    while the C code runs)."""
    import concurrent.futures as cf
    import numpy as np
    import oracle
    from paper_1608_00099_amd import inputs
    single_bytes, single_s = 0, 0.0
    par_bytes, par_s = 0, [0.0, 0.0, 0.0]
    pool = cf.ThreadPoolExecutor(max_workers=threads)

    def run_par(calls):
        parts = [calls[t::threads] for t in range(threads)]
        t0 = time.perf_counter()
        list(pool.map(lambda cs: [c() for c in cs], parts))
        return time.perf_counter() - t0

    for d in range(2, 9):
        src_s, dst_s = inputs.cfg2_pad_shapes(d, log2_target)
        src = inputs.uniform(2, src_s, 90, d).reshape(-1)
        dst = np.zeros(prod(dst_s), dtype=np.float32)
        t0 = time.perf_counter()
        oracle.copy(src_s, dst, dst_s, src, src_s)
        single_s += time.perf_counter() - t0
        single_bytes += 8 * prod(src_s)
        calls = [(lambda sub=sub, b=b: oracle.copy(sub, dst, dst_s, src, src_s, b[0], b[1]))
                 for sub, b in _slabs(src_s, [dst_s, src_s], [0, 0], 4 * threads)]
        for r in range(3):
            par_s[r] += run_par(calls)
        par_bytes += 8 * prod(src_s)
        del src, dst, calls
        xs, ys, zs = inputs.cfg2_inter_shapes(d, log2_target)
        x = inputs.uniform(2, xs, 91, d).reshape(-1)
        y = inputs.uniform(2, ys, 92, d).reshape(-1)
        z = inputs.uniform(2, zs, 93, d).reshape(-1)
        t0 = time.perf_counter()
        oracle.mul_acc(xs, x, xs, y, ys, z, zs)
        single_s += time.perf_counter() - t0
        single_bytes += 16 * prod(xs)
        calls = [(lambda sub=sub, b=b: oracle.mul_acc(sub, x, xs, y, ys, z, zs, b[0], b[1], b[2]))
                 for sub, b in _slabs(xs, [xs, ys, zs], [0, 0, 0], 4 * threads)]
        for r in range(3):
            par_s[r] += run_par(calls)
        par_bytes += 16 * prod(xs)
        del x, y, z, calls
        log("cpu oracle d=%d done (%.1f s single, %.1f s threaded so far)"
            % (d, single_s, sum(par_s)))
    pool.shutdown()
    par = sorted(par_bytes / t / 1e9 for t in par_s)
    return {"single": (single_bytes / single_s / 1e9, single_s),
            "threaded": (par[1], par[0], par[2], sum(par_s))}


def host_cpus():
    """CPUs this process may run on (what nproc reports)."""
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def cpu_info():
    """The host CPU as lscpu and /proc/cpuinfo describe it: model name,
    family/model/stepping, logical CPUs available, threads per core, clock."""
    info = {"cpus": host_cpus()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and "model" not in info:
                    info["model"] = v
                elif k == "cpu family" and "family" not in info:
                    info["family"] = int(v)
                elif k == "model" and "model_id" not in info:
                    info["model_id"] = int(v)
                elif k == "stepping" and "stepping" not in info:
                    info["stepping"] = v
                elif k == "cpu MHz" and "mhz" not in info:
                    info["mhz"] = float(v)
                elif k == "bogomips" and "bogomips" not in info:
                    info["bogomips"] = float(v)
                elif k == "siblings" and "siblings" not in info:
                    info["siblings"] = int(v)
                elif k == "cpu cores" and "cores_per_socket" not in info:
                    info["cores_per_socket"] = int(v)
    except (OSError, ValueError):
        pass
    if "siblings" in info and "cores_per_socket" in info and info["cores_per_socket"]:
        info["threads_per_core"] = info["siblings"] // info["cores_per_socket"]
    return info


def cpu_model():
    i = cpu_info()
    s = i.get("model", "unknown CPU")
    if "family" in i:
        s += " (family %d model %d stepping %s)" % (i["family"], i.get("model_id", -1),
                                                    i.get("stepping", "?"))
    s += ", %d CPUs" % i["cpus"]
    if "mhz" in i:
        s += " at %.0f MHz" % i["mhz"]
    return s


def _moment_names(d, cov):
    names = ["M"] + ["E%d" % i for i in range(d)]
    if cov:
        names += ["C%d%d" % (i, j) for i in range(d) for j in range(i, d)]
    return names


def _per_result_error(got32, ref, d, cov):
    """|g - o| / |o| per result (M, every E_i, every C_ij); an entry whose
    float64 value is exactly 0 is judged by its absolute error against
    the scale max(1, max_i C_ii)."""
    import numpy as np
    got = np.asarray(got32, dtype=np.float64)
    n = len(got)
    ref = np.asarray(ref, dtype=np.float64)[:n]
    scale = 1.0
    if cov and d:
        scale = max(1.0, max(abs(ref[1 + d + i * d - i * (i - 1) // 2]) for i in range(d)))
    out = {}
    for name, g, o in zip(_moment_names(d, cov), got, ref):
        out[name] = abs(g - o) / abs(o) if o != 0 else abs(g - o) / scale
    return out


def moments_errors(dev):
    """The float32 moments of the library against the float64 oracle, per
    result: cfg3 (16^6 PMF, M, E and the covariance: 28 results) and the
    moments step of cfg5's pipeline (the E-based loss reads M and E: 6
    results), each on the same float32 weights."""
    import numpy as np
    import torch
    import oracle
    from paper_1608_00099_amd import api, inputs
    res = {}
    p_np = inputs.cfg3_values()
    p = torch.from_numpy(p_np).to(dev)
    o32, _ = api.moments(p, cov=True)
    t0 = time.perf_counter()
    ref = oracle.moments(inputs.CFG3_SHAPE, [p_np.reshape(-1)], [inputs.CFG3_SHAPE], cov=True)
    t_or = time.perf_counter() - t0
    e = _per_result_error(o32.cpu().numpy(), ref, 6, True)
    res["cfg3_16pow6_cov"] = {"max": max(e.values()), "per_result": e,
                              "oracle_seconds": round(t_or, 3)}
    x_np, w_np, _ = inputs.cfg5_values()
    P = api.pad_embed(torch.from_numpy(x_np).to(dev), inputs.CFG5_P)
    y = api.mul(P, torch.from_numpy(w_np).to(dev))
    o32, _ = api.moments(y, cov=False)
    y_np = y.cpu().numpy()
    ref = oracle.moments(inputs.CFG5_W, [y_np.reshape(-1)], [inputs.CFG5_W], cov=False)
    e = _per_result_error(o32.cpu().numpy(), ref, 5, False)
    res["cfg5_pipeline_first"] = {"max": max(e.values()), "per_result": e}
    del p, P, y
    return res


# ---------------------------------------------------------------------------
# Extras: the other configurations of the hot path
# ---------------------------------------------------------------------------

def event_ms(fn, reps=10, warm=2, pre=None, cover=True):
    """Median/min/max ms of fn between HIP events.  `pre` (e.g. a cache
    flush) runs before every timed call; otherwise an untimed call of fn
    covers the host's enqueue latency (cover=False: fn alone, host-bound)."""
    import torch
    s = torch.cuda.current_stream()
    for _ in range(warm):
        if pre:
            pre()
        fn()
    ms = []
    for _ in range(reps):
        if pre:
            pre()
        elif cover:
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    ms.sort()
    return {"median_ms": ms[len(ms) // 2], "min_ms": ms[0], "max_ms": ms[-1]}


def wall_ms(fn, n=20):
    """Host wall time per call of fn over n back-to-back calls (the device
    drained before and after): what a loop calling fn sustains, enqueue
    overhead included."""
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / n * 1e3


def graph_ms(fn, reps=10):
    """GPU time of fn's launches captured once in a torch CUDA graph and
    replayed (no host work between the kernels)."""
    import torch
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    t = event_ms(g.replay, reps=reps, warm=1)
    del g
    return t


EXTRAS = ("ceiling", "cfg1", "cfg3", "cfg4", "cfg5", "paper", "reduce", "fftconv")


def extras(dev, only=None):
    """The secondary configurations (all of them, or only `only`)."""
    import torch
    out = {}
    want = (lambda k: only is None or only == k)
    # 1 GiB streaming-copy ceiling (torch's device copy); its destination is
    # the scratch written between cold runs (>= 1 GiB beats the 256 MB cache)
    n = 1 << 28
    flush = torch.empty(n, dtype=torch.float32, device=dev)
    if want("ceiling"):
        a = torch.empty(n, dtype=torch.float32, device=dev).fill_(1.0)
        t = event_ms(lambda: flush.copy_(a))
        out["copy_ceiling"] = {"GBs": 2 * 4 * n / t["median_ms"] / 1e6, "bytes": 8 * n,
                               "what": "torch device copy of 1 GiB"}
        del a
        log("ceiling done")
    if want("cfg1"):
        _cfg1(dev, out)
    if want("cfg3"):
        _cfg3(dev, flush, out)
    if want("cfg4"):
        _cfg4(dev, out)
    if want("cfg5"):
        _cfg5(dev, out)
    if want("paper"):
        _paper(dev, flush, out)
    if want("reduce"):
        _reduce(dev, flush, out)
    if want("fftconv"):
        _fftconv(dev, out)
    return out


def _read_flush(flush):
    """A read over the 1 GiB scratch: evicts the caches like the write does,
    but leaves no dirty lines whose write-back would compete with the next
    kernel's reads."""
    return lambda: flush.sum()


def _cold_warm(fn, flush, nbytes):
    """Median GPU time of fn after a 1 GiB write (cold), after a 1 GiB read
    (cold_clean: the same eviction without dirty lines left in the
    memory-side cache) and right after itself (warm), with the effective
    GB/s of nbytes."""
    c = event_ms(fn, pre=lambda: flush.fill_(0.0))
    cc = event_ms(fn, pre=_read_flush(flush))
    w = event_ms(fn)
    return {"cold": dict(c, GBs=nbytes / c["median_ms"] / 1e6),
            "cold_clean": dict(cc, GBs=nbytes / cc["median_ms"] / 1e6),
            "warm": dict(w, GBs=nbytes / w["median_ms"] / 1e6), "bytes": nbytes}


def _paper(dev, flush, out):
    """The paper's four benchmarks (Section 3) at its shapes (benchmarks 1
    and 3 with the library autotuner's schedule, the default schedule's
    figures beside them)."""
    import torch
    from paper_1608_00099_amd import api
    from paper_1608_00099_amd import _lib as L
    big, small = (1 << 10, 1 << 9, 1 << 8), (1 << 9, 1 << 9, 1 << 5)
    # benchmark 1: crop (2^10, 2^9, 2^8) -> (2^9, 2^9, 2^5), float32 and float64
    for dt, name in ((torch.float32, "f32"), (torch.float64, "f64")):
        a = torch.rand(big, dtype=dt, device=dev)
        o = torch.empty(small, dtype=dt, device=dev)
        nb = 2 * prod(small) * a.element_size()
        fn = (lambda: api.copy_(o, a, counter=small))
        default = _cold_warm(fn, flush, nb)
        # the library's autotuner on this crop, then the same measurement
        api.autotune(L.OP_COPY, [o, a], counter=small, params=L.CopyParams(a.element_size()))
        out["paper_b1_crop_" + name] = dict(_cold_warm(fn, flush, nb), default_schedule=default)
        del a, o
    # benchmark 2: inner product over the shared tuples
    a = torch.rand(big, dtype=torch.float32, device=dev)
    b = torch.rand(small, dtype=torch.float32, device=dev)
    out["paper_b2_dot"] = _cold_warm(lambda: api.dot(a, b), flush, 8 * prod(small))
    del a, b
    # benchmark 3: x <- x + y*x - z at the paper's shapes
    xs, ys, zs = (129, 32, 13, 16), (253, 64, 64, 23), (256, 39, 64, 33)
    x = torch.rand(xs, device=dev)
    y = torch.rand(ys, device=dev)
    z = torch.rand(zs, device=dev)
    default = _cold_warm(lambda: api.xpyx_mz_(x, y, z), flush, 16 * prod(xs))
    api.autotune(L.OP_XPYX_MZ, [x, y, z])
    out["paper_b3_update"] = dict(_cold_warm(lambda: api.xpyx_mz_(x, y, z), flush, 16 * prod(xs)),
                                  default_schedule=default)
    del x, y, z
    # benchmark 4: naive convolution of two (2^8, 2^3) float64 matrices
    l = torch.rand((256, 8), dtype=torch.float64, device=dev)
    r = torch.rand((256, 8), dtype=torch.float64, device=dev)
    o = torch.empty((511, 15), dtype=torch.float64, device=dev)
    t = event_ms(lambda: api.conv(l, r, out=o), reps=20)
    macs = prod((256, 8)) * prod((256, 8))
    out["paper_b4_conv"] = dict(t, multiply_adds=macs,
                                GFLOPs=2 * macs / t["median_ms"] / 1e6)
    log("paper benchmarks done")


def _reduce(dev, flush, out):
    """Marginalization and the nonzero bounding box over the 16^6 PMF."""
    import torch
    from paper_1608_00099_amd import api, inputs
    p = torch.from_numpy(inputs.cfg3_values()).to(dev)
    nb = 4 * p.numel()
    out["marginal_16pow6_keep0"] = _cold_warm(lambda: api.marginal(p, (1, 0, 0, 0, 0, 0)), flush,
                                              nb)
    out["marginal_16pow6_keep5"] = _cold_warm(lambda: api.marginal(p, (1, 1, 1, 1, 1, 0)), flush,
                                              nb)
    sparse = torch.where(torch.rand_like(p) < 1e-3, p, torch.zeros_like(p))
    out["bbox_16pow6"] = _cold_warm(lambda: api.bbox(sparse), flush, nb)
    out["dot_16pow6_2ops"] = _cold_warm(lambda: api.dot(p, sparse), flush, 2 * nb)
    log("reductions done")


def _fftconv(dev, out):
    """FFT convolution of a batch of 3-d pairs: the share of the zero-pads and
    the crop (this library's kernels) against the transforms."""
    import torch
    from paper_1608_00099_amd import api, fftconv
    B, sx, sy = 64, (48, 48, 48), (16, 16, 16)
    x = torch.rand((B,) + sx, device=dev)
    y = torch.rand((B,) + sy, device=dev)
    s = fftconv.conv_shape(sx, sy)
    n = tuple(fftconv.good_size(v) for v in s)
    # the library's autotuner on the two pads and the crop
    from paper_1608_00099_amd import _lib as L
    full = torch.empty((B,) + n, device=dev)
    cropped = torch.empty((B,) + s, device=dev)
    api.autotune(L.OP_EMBED_FILL, [full, x], params=L.CopyParams(4))
    api.autotune(L.OP_EMBED_FILL, [full, y], params=L.CopyParams(4))
    api.autotune(L.OP_COPY, [cropped, full], counter=(B,) + s, params=L.CopyParams(4))
    del cropped
    fftconv.fft_conv(x, y, batch_dims=1)          # plans the transforms
    t_all = event_ms(lambda: fftconv.fft_conv(x, y, batch_dims=1), reps=10)
    xp = api.pad_embed(x, (B,) + n)
    yp = api.pad_embed(y, (B,) + n)
    t_pad = event_ms(lambda: (api.pad_embed(x, (B,) + n), api.pad_embed(y, (B,) + n)), reps=10)
    t_crop = event_ms(lambda: api.crop(full, (B,) + s), reps=10)
    pad_bytes = 4 * B * (prod(sx) + prod(sy) + 2 * prod(n))
    crop_bytes = 8 * B * prod(s)
    out["fftconv_b64_48c_16c"] = {
        "total": t_all, "pads": dict(t_pad, GBs=pad_bytes / t_pad["median_ms"] / 1e6),
        "crop": dict(t_crop, GBs=crop_bytes / t_crop["median_ms"] / 1e6),
        "pad_crop_share": (t_pad["median_ms"] + t_crop["median_ms"]) / t_all["median_ms"],
        "fft_shape": list(n)}
    del xp, yp, full
    log("fft convolution done")


def _cfg1(dev, out):
    import torch
    from paper_1608_00099_amd import api, inputs
    # cfg1: small pad-embed (launch-latency bound)
    src = torch.from_numpy(inputs.cfg1_values()).to(dev)
    dst = torch.zeros(inputs.CFG1_DST, dtype=torch.float32, device=dev)
    nb = 8 * prod(inputs.CFG1_SRC)
    t = graph_ms(lambda: [api.pad_embed_into(dst, src) for _ in range(100)], reps=10)
    per = t["median_ms"] / 100
    out["cfg1_pad_embed"] = {"ms_per_launch": per, "GBs": nb / per / 1e6, "bytes": nb,
                             "cache": "warm", "timing": "100 launches captured in one graph"}


def _cfg3(dev, flush, out):
    import torch
    from paper_1608_00099_amd import api, inputs
    # cfg3: moments of a 16^6 PMF (64 MiB: cold runs flush the cache first)
    p = torch.from_numpy(inputs.cfg3_values()).to(dev)
    nb = 4 * p.numel()
    o32, o64 = api.moments(p, cov=True)
    t_cold = event_ms(lambda: api.moments(p, cov=True), pre=lambda: flush.fill_(0.0))
    t_clean = event_ms(lambda: api.moments(p, cov=True), pre=_read_flush(flush))
    t_warm = event_ms(lambda: api.moments(p, cov=True))
    out["cfg3_moments_cov"] = {"cold": dict(t_cold, GBs=nb / t_cold["median_ms"] / 1e6),
                               "cold_clean": dict(t_clean, GBs=nb / t_clean["median_ms"] / 1e6),
                               "warm": dict(t_warm, GBs=nb / t_warm["median_ms"] / 1e6),
                               "bytes": nb}
    log("moments done")



def _cfg4(dev, out):
    import torch
    from paper_1608_00099_amd import api, inputs
    from paper_1608_00099_amd import _lib as L
    # cfg4: 4096 ragged pads for FFT convolution, one persistent graph launch
    shapes = inputs.cfg4_shapes()
    xs = [torch.from_numpy(x).to(dev) for x in inputs.cfg4_values(shapes)]
    dsts = [torch.empty(inputs.padded_shape(sx, sy), dtype=torch.float32, device=dev)
            for sx, sy in shapes]
    nb = sum(4 * d_.numel() + 4 * x.numel() for d_, x in zip(dsts, xs))
    items = [[d_, x] for d_, x in zip(dsts, xs)]
    batch = api.Batch()
    t0 = time.perf_counter()
    batch.apply(L.OP_EMBED_FILL, items)          # plan, upload, capture, launch
    torch.cuda.synchronize()
    t_plan = (time.perf_counter() - t0) * 1e3
    t_def = event_ms(batch.launch, reps=20)      # replay, the library's default schedule
    info_def = dict(batch.info(), schedule=batch.schedule())
    # the batch autotuner picks the schedule of this batch (cold timing of
    # the candidates), then the batch is planned and captured again with it
    t0 = time.perf_counter()
    batch.autotune(L.OP_EMBED_FILL, items)
    t_tune = time.perf_counter() - t0
    batch.apply(L.OP_EMBED_FILL, items)
    torch.cuda.synchronize()
    t_b = event_ms(batch.launch, reps=20)        # replay of the captured launch
    info = dict(batch.info(), schedule=batch.schedule(), tune_seconds=round(t_tune, 2))
    t_pe = event_ms(lambda: [api.embed_fill_(d_, x) for d_, x in zip(dsts, xs)], reps=3, warm=1,
                    cover=False)
    t_pg = graph_ms(lambda: [api.embed_fill_(d_, x) for d_, x in zip(dsts, xs)], reps=5)
    out["cfg4_batched_pad"] = {
        "batched": dict(t_b, GBs=nb / t_b["median_ms"] / 1e6, **info),
        "batched_default_schedule": dict(t_def, GBs=nb / t_def["median_ms"] / 1e6,
                                         first_call_ms=t_plan, **info_def),
        "plain_per_item_eager": dict(t_pe, GBs=nb / t_pe["median_ms"] / 1e6, launches=len(items)),
        "plain_per_item_graph": dict(t_pg, GBs=nb / t_pg["median_ms"] / 1e6, launches=len(items)),
        "speedup_vs_plain_eager": t_pe["median_ms"] / t_b["median_ms"],
        "speedup_vs_plain_graph": t_pg["median_ms"] / t_b["median_ms"],
        "bytes": nb, "items": len(items)}
    batch.close()
    del xs, dsts, items
    log("batched done")


def _tune_cfg5(dev, xd, wd):
    """The library's autotuner on each element-wise launch of the pipeline
    (pad-embed, product, product adjoint, crop), on buffers of the
    pipeline's shapes: every later call with the same shapes (the raw,
    autograd and graphed steps below) runs with the tuned schedule.  The
    moments kernels have one schedule."""
    import torch
    from paper_1608_00099_amd import api, inputs
    from paper_1608_00099_amd import _lib as L
    P = torch.empty(inputs.CFG5_P, device=dev)
    y = torch.empty(inputs.CFG5_W, device=dev)
    gy = torch.rand(inputs.CFG5_W, device=dev)
    ga = torch.empty_like(P)
    gb = torch.empty_like(wd)
    gx = torch.empty_like(xd)
    probs = {"pad_embed": (L.OP_EMBED_FILL, [P, xd], dict(params=L.CopyParams(4))),
             "mul": (L.OP_MUL, [y, P, wd], dict(counter=inputs.CFG5_W)),
             "mul_adj": (L.OP_MUL_ADJ, [ga, gb, gy, P, wd], {}),
             "crop": (L.OP_COPY, [gx, ga], dict(counter=inputs.CFG5_X, params=L.CopyParams(4)))}
    out = {}
    for name, (op, ts, kw) in probs.items():
        api.autotune(op, ts, **kw)
        out[name] = api.schedule_get(op, ts, **kw)
    del P, y, gy, ga, gb, gx
    return out


def _cfg5(dev, out):
    import numpy as np
    import torch
    from paper_1608_00099_amd import api, autograd, inputs
    # cfg5: differentiable pipeline, autograd vs the raw kernels
    x_np, w_np, lam_np = inputs.cfg5_values()
    x = torch.from_numpy(x_np).to(dev).requires_grad_(True)
    w = torch.from_numpy(w_np).to(dev).requires_grad_(True)
    lam = torch.from_numpy(lam_np.astype(np.float32)).to(dev)
    tuned = _tune_cfg5(dev, x.detach(), w.detach())

    def fwd_bwd():
        # a fresh step: gradients set to None, as optimizers' zero_grad does,
        # so backward writes them instead of adding a second full pass
        x.grad = None
        w.grad = None
        P = autograd.pad_embed(x, inputs.CFG5_P)
        y = autograd.mul(P, w)
        M, E, C = autograd.moments(y)
        loss = (lam * E).sum()
        loss.backward()
        return loss

    t_auto = event_ms(fwd_bwd, reps=10)
    xd, wd = x.detach(), w.detach()

    def raw():
        P = api.pad_embed(xd, inputs.CFG5_P)
        y = api.mul(P, wd)
        o32, o64 = api.moments(y, cov=False, cached=True)
        gm = torch.zeros(1 + 5, dtype=torch.float32, device=dev)
        gy = api.moments_adj(inputs.CFG5_W, o64, gm, cov=False)
        gP, gw = api.mul_adj(gy, P, wd)
        api.crop(gP, inputs.CFG5_X)

    t_raw = event_ms(raw, reps=10)

    # the same step, forward and backward captured as one graph over the
    # leaf tensors themselves (no static-input copies) and replayed
    xg, wg = xd.clone().requires_grad_(True), wd.clone().requires_grad_(True)

    def step(a, b):
        P = autograd.pad_embed(a, inputs.CFG5_P)
        y = autograd.mul(P, b)
        M, E, C = autograd.moments(y)
        return (lam * E).sum()

    cap = autograd.CapturedStep(step, (xg, wg))
    t_graph = event_ms(cap.replay, reps=10)
    t_graph["wall_ms_per_step"] = wall_ms(cap.replay)
    t_auto["wall_ms_per_step"] = wall_ms(fwd_bwd)
    t_raw["wall_ms_per_step"] = wall_ms(raw)
    del cap
    fwd_bytes = (4 * prod(inputs.CFG5_P) + 4 * prod(inputs.CFG5_X) + 12 * prod(inputs.CFG5_W)
                 + 4 * prod(inputs.CFG5_W))
    bwd_bytes = (4 * prod(inputs.CFG5_W) + 20 * prod(inputs.CFG5_W)
                 + 4 * (prod(inputs.CFG5_P) - prod(inputs.CFG5_W)) + 8 * prod(inputs.CFG5_X))
    out["cfg5_autograd"] = {"autograd_fwd_bwd": t_auto, "raw_kernels": t_raw,
                            "autograd_graphed": t_graph,
                            "autograd_over_raw": t_auto["median_ms"] / t_raw["median_ms"],
                            "graphed_over_raw": t_graph["median_ms"] / t_raw["median_ms"],
                            "GBs_raw": (fwd_bytes + bwd_bytes) / t_raw["median_ms"] / 1e6,
                            "bytes": fwd_bytes + bwd_bytes, "schedules": tuned}
    log("autograd done")


def load_traffic(kernel, src_hash):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    e = t.get(kernel)
    if not e or e.get("source_hash") != src_hash:
        return None
    return e.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--only", choices=EXTRAS, default=None,
                    help="time one secondary configuration alone (for profiling)")
    ap.add_argument("--schedules", default=SCHEDULES,
                    help="JSON of the launch schedules to pin (launch name -> schedule), "
                         "written by --retune --save-schedules")
    ap.add_argument("--retune", action="store_true",
                    help="ignore --schedules: run the autotuner on every launch, then refine "
                         "the schedules in sequence")
    ap.add_argument("--no-seq-tune", action="store_true",
                    help="with --retune: the library's autotuner per launch only")
    ap.add_argument("--save-schedules", default=None,
                    help="write the schedules the sweep ran with to this JSON file")
    ap.add_argument("--no-tune", action="store_true",
                    help="the library's default schedules (no pinning, no tuning)")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="threads of the threaded CPU oracle timing (default: every CPU this "
                         "process may use, as nproc reports)")
    ap.add_argument("--cpu-log2", type=float, default=26,
                    help="log2 elements per tensor of the CPU oracle sample")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_1608_00099_amd import _lib as L
    L.lib()
    dev = torch.device("cuda:0")
    if args.only:
        print(json.dumps({"only": args.only, "extras": extras(dev, args.only)}), flush=True)
        return
    log("allocating the d=2..8 sweep")
    sw = Sweep(dev)
    launches = sw.launches()
    if args.no_tune:
        how = "library defaults"
    elif args.retune or not os.path.exists(args.schedules):
        if args.no_seq_tune:
            log("autotuning the %d launch schedules" % len(launches))
            autotune_all(launches)
            how = "autotuned per launch"
        else:
            log("ranking schedules alone, then refining them in sequence")
            sequence_tune(launches, dev)
            how = "ranked alone over a grid, refined in sequence"
    else:
        pin_schedules(launches, args.schedules)
        how = "pinned from %s" % os.path.relpath(args.schedules, ROOT)
    if args.save_schedules:
        save_schedules(launches, args.save_schedules)
    tuned = tuned_summary(launches)
    step_bytes = sum(x[3] for x in launches)
    fns = [x[2] for x in launches]
    log("timing %d steps after %d warm-up steps" % (args.steps, args.warmup))
    ms_step, wall_ms = time_steps_plain(fns, args.steps, args.warmup)
    value = step_bytes / (ms_step * 1e-3) / 1e9
    log("step %.3f ms, %.1f GB/s" % (ms_step, value))
    # The same number of steps again, with HIP events between the launches:
    # each kernel's duration in the sequence (after a different kernel over
    # other buffers, as in use).  The markers lengthen this pass slightly;
    # `value` comes from the pass above.
    ms_instr, _, per = time_steps(fns, args.steps, 1)
    log("instrumented step %.3f ms" % ms_instr)

    # Per-launch durations (inside the instrumented steps) and the dominant
    # kernel's roofline.
    per_op = {}
    by_kernel = {}
    for (name, op, fn, nbytes, it), ts in zip(launches, per):
        plan, kname = plan_of(op, it)
        avg = sum(ts) / len(ts)
        per_op[name] = {"ms": avg, "ms_min": min(ts), "ms_max": max(ts),
                        "GBs": nbytes / avg / 1e6, "bytes": nbytes, "kernel": kname,
                        "box_rows": plan["box_rows"], "units": plan["units"]}
        k = by_kernel.setdefault(kname, {"ms": 0.0, "bytes": 0, "launches": 0})
        k["ms"] += avg
        k["bytes"] += nbytes
        k["launches"] += 1
    dom = max(by_kernel, key=lambda k: by_kernel[k]["ms"])
    dk = by_kernel[dom]
    avg_ms = dk["ms"] / dk["launches"]
    avg_bytes = dk["bytes"] / dk["launches"]
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    src_hash = kernel_source_hash()
    traffic = load_traffic(dom, src_hash)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                "traffic": traffic, "kernel": dom, "launches_per_step": dk["launches"],
                "avg_launch_ms": round(avg_ms, 5), "algorithmic_bytes_per_launch": int(avg_bytes)}

    # The pad-embed destinations are zeroed once, at allocation; a zero
    # fill of all seven (torch's fill kernel) is timed on its own line, not
    # folded into the step.
    zbytes = sum(4 * it["dst"].numel() for it in sw.items)
    tz = event_ms(lambda: [it["dst"].zero_() for it in sw.items], reps=5)
    zero_fill = {"ms": round(tz["median_ms"], 4), "bytes": zbytes,
                 "GBs": round(zbytes / tz["median_ms"] / 1e6, 1),
                 "what": "zero fill of the seven pad-embed destinations, not part of the step"}

    cpu = None
    if not args.no_cpu:
        threads = host_cpus() if args.cpu_threads <= 0 else max(1, min(args.cpu_threads,
                                                                         host_cpus()))
        log("CPU oracle baseline (2^%g elements per tensor, 1 and %d threads)"
            % (args.cpu_log2, threads))
        r = cpu_baseline(args.cpu_log2, threads)
        gbs1, secs1 = r["single"]
        med, lo, hi, secs_t = r["threaded"]
        cpu = {"value": round(med, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
               "sample": "the same d=2..8 copy + x+=y*z recipe at 2^%g elements per tensor "
                         "(the full step at 2^26), C oracle on %s: %d threads each taking "
                         "windows of the leading counter axes, median of 3 passes (%.1f s in "
                         "all)" % (args.cpu_log2, cpu_model(), threads, secs_t),
               "min": round(lo, 3), "max": round(hi, 3),
               "single_thread": {"value": round(gbs1, 3), "cores": 1,
                                 "seconds": round(secs1, 2)},
               "host": cpu_info()}
        log("moments per-result error against the float64 oracle")
        cpu["moments_error"] = moments_errors(dev)

    ext = None
    if not args.no_extras:
        ext = extras(dev)

    line = {
        "metric": "effective HBM GB/s & % of peak; batched/autograd vs plain kernels, same GPU",
        "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "runtime-dimension sweep d=2..8, ~2^26 float32 elements per tensor: "
                               "pad-embed (+1..16 per axis) and x+=y*z over the intersection of "
                               "three shapes",
                   "bytes_per_step": step_bytes, "pct_of_peak": round(100 * value / PEAK_HBM_GBS, 2),
                   "wall_ms_per_step": round(wall_ms, 4),
                   "instrumented_ms_per_step": round(ms_instr, 4)},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "dst_zero_fill": zero_fill,
        "per_op": per_op,
        "tuned": tuned,
        "schedules": how,
        "extras": ext,
        "kernel_source": src_hash,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
