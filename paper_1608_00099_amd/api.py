"""Torch-facing helpers over the C ABI.

PyTorch supplies device memory and the current stream; every step of the
computation runs in libtriot's kernels.  Operands are contiguous CUDA/HIP
tensors viewed as row-major parent buffers; ``shape`` and ``base`` arguments
describe windows into them (Section 4 of the paper: slices with a bias).
"""
from __future__ import annotations

import threading

import torch

from . import _lib as L
from ._lib import TriotError

_ws_lock = threading.Lock()
_ws_cache: dict = {}


def _stream(dev: torch.device):
    return torch.cuda.current_stream(dev).cuda_stream


def _check(st: int, what: str):
    if st != L.OK:
        raise TriotError(st, what)


def _prep(tensors, shapes):
    dev = None
    for t in tensors:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError("triot operands must be GPU tensors")
        if not t.is_contiguous():
            raise ValueError("triot operands must be contiguous parent buffers")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError("all operands must live on one device")
    if shapes is None:
        shapes = [tuple(t.shape) for t in tensors]
    return dev, [tuple(int(v) for v in s) for s in shapes]


def _ptr(t):
    return t.data_ptr() if (t is not None and t.numel() > 0) else 0


def apply(op, tensors, shapes=None, counter=None, bases=None, params=None, out=None,
          workspace=None, what="triot_apply"):
    """Run one co-iteration on the current stream (see include/triot.h)."""
    dev, shapes = _prep(tensors, shapes)
    d = len(shapes[0]) if shapes else 0
    if any(len(s) != d for s in shapes):
        raise ValueError("all operand shapes must have the same dimension")
    ws_ptr, ws_bytes = 0, 0
    if workspace is not None:
        ws_ptr, ws_bytes = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    st = L.triot_apply(op, len(tensors), d, shapes, counter, [_ptr(t) for t in tensors], bases,
                       params, out.data_ptr() if out is not None else 0, ws_ptr, ws_bytes,
                       _stream(dev))
    _check(st, what)


def workspace_for(op, shapes, counter, dev):
    """A zero-initialised workspace, cached per (device, stream, size)."""
    d = len(shapes[0]) if shapes else 0
    nbytes = L.triot_workspace_size(op, len(shapes), d, shapes, counter)
    if nbytes == 0:
        return None
    key = (dev, _stream(dev))
    with _ws_lock:
        ws = _ws_cache.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.zeros(max(nbytes, 4096), dtype=torch.uint8, device=dev)
            _ws_cache[key] = ws
    return ws


# ---------------------------------------------------------------------------
# Copies: zero-pad embedding and crop (Sections 1 and 3)
# ---------------------------------------------------------------------------

def _elem_params(t):
    es = t.element_size()
    if es not in (4, 8):
        raise ValueError("copies move 4- or 8-byte elements")
    return L.CopyParams(es)


def copy_(dst, src, counter=None, dst_shape=None, src_shape=None, dst_base=0, src_base=0):
    """dst[t] = src[t] for every tuple of ``counter`` (default: the shapes'
    intersection)."""
    if dst.element_size() != src.element_size():
        raise ValueError("element sizes differ")
    shapes = [tuple(dst_shape or dst.shape), tuple(src_shape or src.shape)]
    apply(L.OP_COPY, [dst, src], shapes, counter, [dst_base, src_base], _elem_params(dst),
          what="copy")
    return dst


def pad_embed_into(dst, x):
    """Zero-pad embedding of x at the origin of a pre-zeroed dst (counter =
    x's shape); only the counter points are written."""
    return copy_(dst, x, counter=tuple(x.shape))


def embed_fill_(dst, src, dst_shape=None, src_shape=None, src_base=0):
    """Over all of dst: src where the tuple lies in src, +0.0 elsewhere."""
    shapes = [tuple(dst_shape or dst.shape), tuple(src_shape or src.shape)]
    apply(L.OP_EMBED_FILL, [dst, src], shapes, None, [0, src_base], _elem_params(dst),
          what="embed_fill")
    return dst


def pad_embed(x, shape):
    """A new tensor of ``shape`` holding x at the origin and zeros elsewhere,
    written in one pass (the zero padding ahead of an FFT convolution)."""
    out = torch.empty(tuple(shape), dtype=x.dtype, device=x.device)
    return embed_fill_(out, x)


def crop(x, shape):
    """A new tensor with x's leading ``shape`` window (benchmark 1's copy)."""
    out = torch.empty(tuple(shape), dtype=x.dtype, device=x.device)
    return copy_(out, x, counter=tuple(shape))


# ---------------------------------------------------------------------------
# Element-wise products over shared tuples
# ---------------------------------------------------------------------------

def _f32(*ts):
    for t in ts:
        if t.dtype != torch.float32:
            raise ValueError("arithmetic ops take float32 tensors")


def mul_acc_(x, y, z, counter=None, shapes=None, bases=None):
    """x[t] += y[t]*z[t] (two roundings) over counter (default: intersection)."""
    _f32(x, y, z)
    apply(L.OP_MUL_ACC, [x, y, z], shapes, counter, bases, what="mul_acc")
    return x


def mul_into(out, a, b, counter=None, shapes=None, bases=None):
    _f32(out, a, b)
    apply(L.OP_MUL, [out, a, b], shapes, counter, bases, what="mul")
    return out


def mul(a, b, counter=None):
    """out[t] = a[t]*b[t] over counter (default: the shapes' intersection)."""
    if counter is None:
        counter = tuple(min(p, q) for p, q in zip(a.shape, b.shape))
    out = torch.empty(tuple(counter), dtype=torch.float32, device=a.device)
    return mul_into(out, a, b, counter=tuple(counter))


def mul_adj(gout, a, b):
    """Adjoint of out = a*b over the intersection I = gout's shape."""
    _f32(gout, a, b)
    ga = torch.empty_like(a)
    gb = torch.empty_like(b)
    apply(L.OP_MUL_ADJ, [ga, gb, gout, a, b], None, None, None, what="mul_adj")
    return ga, gb


# ---------------------------------------------------------------------------
# Index-weighted moments (Algorithm 11) and their adjoint
# ---------------------------------------------------------------------------

def n_moments(d: int, cov: bool) -> int:
    return 1 + d + (d * (d + 1) // 2 if cov else 0)


def moments(p, cov=True, others=(), counter=None, cached=False):
    """(out32, out64): [M, E_0..E_{d-1}(, upper-triangle C)] of the weights
    w(t) = p[t] * prod(others[k][t]) over counter (default: intersection).
    cached: a load hint for operands the previous kernel just wrote (no
    effect on the results)."""
    tensors = [p] + list(others)
    _f32(*tensors)
    dev, shapes = _prep(tensors, None)
    d = p.dim()
    nout = n_moments(d, cov)
    out32 = torch.empty(nout, dtype=torch.float32, device=dev)
    out64 = torch.empty(nout, dtype=torch.float64, device=dev)
    ws = workspace_for(L.OP_MOMENTS, shapes, counter, dev)
    flags = L.MOMENTS_FIRST | (L.MOMENTS_COV if cov else 0) | (L.MOMENTS_CACHED if cached else 0)
    params = L.MomentsParams(flags, out64.data_ptr())
    apply(L.OP_MOMENTS, tensors, shapes, counter, None, params, out=out32, workspace=ws,
          what="moments")
    return out32, out64


def moments_adj(shape, mom64, gmom32, cov=True, device=None):
    """g[t] = d loss / d w(t) for every t of ``shape``."""
    dev = device or mom64.device
    g = torch.empty(tuple(shape), dtype=torch.float32, device=dev)
    gm = gmom32.contiguous()
    params = L.MomentsAdjParams(L.MOMENTS_FIRST | (L.MOMENTS_COV if cov else 0),
                                mom64.data_ptr(), gm.data_ptr())
    apply(L.OP_MOMENTS_ADJ, [g], None, None, None, params, what="moments_adj")
    return g


# ---------------------------------------------------------------------------
# Benchmarks 2-4 of Section 3 and the tuple-reading reductions of Section 2
# ---------------------------------------------------------------------------

def dot(a, b, *others, counter=None):
    """(out32, out64): sum_t a[t] * b[t] * ... over the shared tuples
    (benchmark 2's inner product), float64 accumulation."""
    tensors = [a, b] + list(others)
    _f32(*tensors)
    dev, shapes = _prep(tensors, None)
    out32 = torch.empty(1, dtype=torch.float32, device=dev)
    out64 = torch.empty(1, dtype=torch.float64, device=dev)
    ws = workspace_for(L.OP_DOT, shapes, counter, dev)
    apply(L.OP_DOT, tensors, shapes, counter, None, L.ReduceParams(out64.data_ptr()), out=out32,
          workspace=ws, what="dot")
    return out32, out64


def xpyx_mz_(x, y, z, counter=None, shapes=None, bases=None):
    """x[t] = (x[t] + y[t]*x[t]) - z[t] over counter (default: the
    intersection; benchmark 3), three roundings."""
    _f32(x, y, z)
    apply(L.OP_XPYX_MZ, [x, y, z], shapes, counter, bases, what="xpyx_mz")
    return x


def marginal(p, keep, others=(), counter=None):
    """(out32, out64): sums of w(t) = p[t] * prod(others[k][t]) over the
    counter axes whose keep flag is false; the result has the kept
    counter extents."""
    tensors = [p] + list(others)
    _f32(*tensors)
    dev, shapes = _prep(tensors, None)
    d = p.dim()
    if counter is None:
        counter = tuple(min(s[i] for s in shapes) for i in range(d))
    kshape = tuple(int(c) for c, k in zip(counter, keep) if k)
    mask = 0
    for i, k in enumerate(keep):
        if k:
            mask |= 1 << i
    out32 = torch.empty(kshape, dtype=torch.float32, device=dev)
    out64 = torch.empty(kshape, dtype=torch.float64, device=dev)
    ws = workspace_for(L.OP_MARGINAL, shapes, counter, dev)
    apply(L.OP_MARGINAL, tensors, shapes, counter, None, L.MarginalParams(mask, out64.data_ptr()),
          out=out32, workspace=ws, what="marginal")
    return out32, out64


def bbox(p, *others, counter=None):
    """int64 [d, 2]: per axis, the least and greatest t_i at which every
    operand is nonzero (all -1 when there is none)."""
    tensors = [p] + list(others)
    _f32(*tensors)
    dev, shapes = _prep(tensors, None)
    d = p.dim()
    out = torch.empty((d, 2), dtype=torch.int64, device=dev)
    ws = workspace_for(L.OP_BBOX, shapes, counter, dev)
    apply(L.OP_BBOX, tensors, shapes, counter, None, None, out=out, workspace=ws, what="bbox")
    return out


def conv(lhs, rhs, out=None):
    """Naive convolution (Algorithms 14 and 15), float64, result shape
    lhs.shape + rhs.shape - 1, equal to the paper's loop order bit for bit."""
    if lhs.dtype != torch.float64 or rhs.dtype != torch.float64:
        raise ValueError("conv takes float64 tensors")
    if lhs.dim() != rhs.dim():
        raise ValueError("conv operands must have the same dimension")
    oshape = tuple(a + b - 1 for a, b in zip(lhs.shape, rhs.shape))
    if out is None:
        out = torch.empty(oshape, dtype=torch.float64, device=lhs.device)
    apply(L.OP_CONV, [out, lhs.contiguous(), rhs.contiguous()],
          [oshape, tuple(lhs.shape), tuple(rhs.shape)], None, None, None, what="conv")
    return out


def index(shapes, counter=None, bases=None, device="cuda"):
    """int64 [n, N]: the offset of every counter tuple in every operand."""
    shapes = [tuple(int(v) for v in s) for s in shapes]
    n, d = len(shapes), len(shapes[0])
    if counter is None:
        counter = tuple(min(s[i] for s in shapes) for i in range(d))
    N = 1
    for c in counter:
        N *= int(c)
    out = torch.empty((n, N), dtype=torch.int64, device=device)
    ptrs = [out.data_ptr()] + [0] * (n - 1)
    st = L.triot_apply(L.OP_INDEX, n, d, shapes, counter, ptrs, bases, None, 0, 0, 0,
                       _stream(out.device))
    _check(st, "index")
    return out


# ---------------------------------------------------------------------------
# Batched form and tuning
# ---------------------------------------------------------------------------

class Batch:
    """A batch handle: the planned work table and captured hipGraph of one
    batch of independent co-iterations (replayed while the batch repeats)."""

    def __init__(self):
        st, self._h = L.triot_batch_create()
        _check(st, "batch_create")

    def close(self):
        if self._h:
            L.triot_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def apply(self, op, items, elem_bytes=4):
        """items: list of operand lists (contiguous GPU tensors); each item's
        counter is the op's default (see include/triot.h)."""
        if not items:
            return
        dev = items[0][0].device
        params = L.CopyParams(elem_bytes) if op in (L.OP_COPY, L.OP_EMBED_FILL) else None
        st = L.triot_apply_batched(op, self._marshal(items), params, self._h, _stream(dev))
        _check(st, "apply_batched")

    @staticmethod
    def _marshal(items):
        out = []
        for ops in items:
            shapes = [tuple(t.shape) for t in ops]
            out.append((len(shapes[0]), len(ops), shapes, None, [_ptr(t) for t in ops], None))
        return out

    def set_schedule(self, cache_policy=1, blocks_per_cu=8, box_rows_max=1024, unit_elems=4096,
                     vec_max=4, unit_order=1):
        """Set the launch schedule of this batch (the next apply re-plans and
        re-captures); the defaults are the library's."""
        sch = L.Schedule(vec_max, cache_policy, blocks_per_cu, box_rows_max, unit_elems,
                         unit_order)
        _check(L.triot_batch_set_schedule(self._h, sch), "batch_set_schedule")

    def autotune(self, op, items, elem_bytes=4, cache_path=None):
        """Time candidate schedules of this batch's persistent launch (cold)
        and keep the fastest on this handle (the op runs several times on
        the given buffers)."""
        if not items:
            return
        dev = items[0][0].device
        params = L.CopyParams(elem_bytes) if op in (L.OP_COPY, L.OP_EMBED_FILL) else None
        st = L.triot_batch_autotune(self._h, op, self._marshal(items), params, _stream(dev),
                                    cache_path)
        _check(st, "batch_autotune")

    def schedule(self):
        """The schedule this handle plans with (dict of triot_schedule)."""
        st, sch = L.triot_batch_get_schedule(self._h)
        _check(st, "batch_get_schedule")
        return {f: getattr(sch, f) for f, _ in L.Schedule._fields_}

    def launch(self, device=None):
        """Replay the last planned batch on the current stream (no
        re-validation: the caller keeps the same buffers alive)."""
        dev = device or torch.device("cuda", torch.cuda.current_device())
        _check(L.triot_batch_launch(self._h, _stream(dev)), "batch_launch")

    def info(self):
        st, units, blocks, replayed = L.triot_batch_info(self._h)
        _check(st, "batch_info")
        return {"units": units, "blocks": blocks, "replayed": bool(replayed)}


def autotune(op, tensors, shapes=None, counter=None, bases=None, params=None, cache_path=None):
    """Pick the fastest launch schedule for this exact problem (runs the op
    several times on the given buffers)."""
    dev, shapes = _prep(tensors, shapes)
    d = len(shapes[0])
    st = L.triot_autotune(op, len(tensors), d, shapes, counter, [_ptr(t) for t in tensors], bases,
                          params, 0, 0, 0, _stream(dev), cache_path)
    _check(st, "autotune")


def schedule_set(op, tensors, shapes=None, counter=None, bases=None, params=None, vec_max=4,
                 cache_policy=1, blocks_per_cu=4, box_rows_max=1024, unit_elems=8192,
                 unit_order=0):
    """Pin the launch schedule of this exact problem (every later call with
    the same plan signature uses it until tune_reset)."""
    dev, shapes = _prep(tensors, shapes)
    sch = L.Schedule(vec_max, cache_policy, blocks_per_cu, box_rows_max, unit_elems, unit_order)
    st = L.triot_schedule_set(op, len(tensors), len(shapes[0]), shapes, counter,
                              [_ptr(t) for t in tensors], bases, params, sch)
    _check(st, "schedule_set")


def schedule_get(op, tensors, shapes=None, counter=None, bases=None, params=None):
    """The launch schedule triot_apply uses for this exact problem (pinned,
    tuned or default), as a dict of schedule_set's keyword arguments."""
    dev, shapes = _prep(tensors, shapes)
    st, sch = L.triot_schedule_get(op, len(tensors), len(shapes[0]), shapes, counter,
                                   [_ptr(t) for t in tensors], bases, params)
    _check(st, "schedule_get")
    return {"vec_max": sch.vec_max, "cache_policy": sch.cache_policy,
            "blocks_per_cu": sch.blocks_per_cu, "box_rows_max": sch.box_rows_max,
            "unit_elems": sch.unit_elems, "unit_order": sch.unit_order}


def tune_reset():
    """Forget every tuned or pinned schedule (the defaults apply again)."""
    L.triot_tune_reset()


def describe(op, shapes, counter=None, ptrs=None, bases=None, params=None):
    """The launch plan triot_apply would use (no device work)."""
    shapes = [tuple(int(v) for v in s) for s in shapes]
    if ptrs is None:
        ptrs = [(k + 1) << 40 for k in range(len(shapes))]
    st, info = L.triot_plan_describe(op, len(shapes), len(shapes[0]), shapes, counter, ptrs, bases,
                                     params)
    _check(st, "plan_describe")
    return {"kernel": info.kernel, "dims": info.dims,
            "extents": [info.extents[i] for i in range(info.dims)], "vec": info.vec,
            "high_axes": info.high_axes, "low_axes": info.low_axes, "box_rows": info.box_rows,
            "units": info.units, "blocks": info.blocks, "threads": info.threads,
            "unroll": info.unroll, "inner_unit": info.inner_unit,
            "cache_policy": info.cache_policy, "unit_order": info.unit_order,
            "row_tail": info.row_tail, "n_tensors": len(shapes)}


_CO_OP = {0: 0, 1: 1, 2: 2, 3: 3, 6: 4, 7: 5}   # public op -> kernel template op


def kernel_name(op, plan):
    """The demangled name of the kernel instance a plan launches (as the
    profiler reports it)."""
    if plan["kernel"] == 1:
        cov = "true" if plan.get("cov") else "false"
        dmax = 8 if plan["dims"] <= 8 else 32
        if op == L.OP_MOMENTS:
            dm = plan["dims"] if plan.get("cov") else dmax
            vec = "true" if plan["vec"] == 4 else "false"
            multi = "true" if plan.get("n_tensors", 1) > 1 else "false"
            return "void triot::moments_kernel<%d, %s, %s, %s, true>(triot::SegPlan)" % (
                dm, cov, vec, multi)
        return "void triot::moments_adj_kernel<%d, %s>(triot::SegPlan)" % (dmax, cov)
    rows1 = "true" if plan["box_rows"] == 1 else "false"
    unit = "true" if plan["inner_unit"] else "false"
    cp = 0 if op == L.OP_INDEX else plan["cache_policy"]
    rag = "true" if plan.get("row_tail") else "false"
    return "void triot::coiter_kernel<%d, %d, %d, %s, %s, %d, %s>(triot::CoPlan)" % (
        _CO_OP[op], plan["vec"], plan["unroll"], rows1, unit, cp, rag)
