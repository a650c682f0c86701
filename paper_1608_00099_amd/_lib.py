"""ctypes binding of libtriot.so: the C ABI of include/triot.h, one Python
function per entry point with the same name, arguments marshalled only.

The library is built in-tree (``python -m paper_1608_00099_amd.build``).
There is no fallback: if the library is missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtriot.so")

MAX_D = 32
MAX_TENSORS = 5

# triot_status
OK, E_INVALID, E_DIM, E_BOUNDS, E_ALIAS, E_OVERFLOW, E_WORKSPACE, E_DEVICE, E_UNSUPPORTED = range(9)
STATUS_NAMES = ["OK", "E_INVALID", "E_DIM", "E_BOUNDS", "E_ALIAS", "E_OVERFLOW", "E_WORKSPACE",
                "E_DEVICE", "E_UNSUPPORTED"]

# triot_op
(OP_COPY, OP_EMBED_FILL, OP_MUL_ACC, OP_MUL, OP_MOMENTS, OP_MOMENTS_ADJ, OP_MUL_ADJ, OP_INDEX,
 OP_DOT, OP_XPYX_MZ, OP_MARGINAL, OP_BBOX, OP_CONV) = range(13)

MOMENTS_FIRST = 1
MOMENTS_COV = 2
MOMENTS_CACHED = 4   # load hint: the operands were just written


class CopyParams(ctypes.Structure):
    _fields_ = [("elem_bytes", ctypes.c_int)]


class MomentsParams(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_int), ("out64", ctypes.c_void_p)]


class ReduceParams(ctypes.Structure):
    _fields_ = [("out64", ctypes.c_void_p)]


class MarginalParams(ctypes.Structure):
    _fields_ = [("keep_mask", ctypes.c_uint32), ("out64", ctypes.c_void_p)]


class MomentsAdjParams(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_int), ("mom", ctypes.c_void_p), ("gmom", ctypes.c_void_p)]


class Item(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("n_tensors", ctypes.c_int),
                ("shapes", ctypes.POINTER(ctypes.c_int64)),
                ("counter_shape", ctypes.POINTER(ctypes.c_int64)),
                ("tensors", ctypes.POINTER(ctypes.c_void_p)),
                ("bases", ctypes.POINTER(ctypes.c_int64))]


class PlanInfo(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int), ("dims", ctypes.c_int),
                ("extents", ctypes.c_int64 * MAX_D), ("vec", ctypes.c_int),
                ("high_axes", ctypes.c_int), ("low_axes", ctypes.c_int),
                ("box_rows", ctypes.c_int64), ("units", ctypes.c_int64),
                ("blocks", ctypes.c_int), ("threads", ctypes.c_int), ("unroll", ctypes.c_int),
                ("inner_unit", ctypes.c_int), ("cache_policy", ctypes.c_int),
                ("unit_order", ctypes.c_int), ("row_tail", ctypes.c_int)]


class Schedule(ctypes.Structure):
    _fields_ = [("vec_max", ctypes.c_int), ("cache_policy", ctypes.c_int),
                ("blocks_per_cu", ctypes.c_int), ("box_rows_max", ctypes.c_int),
                ("unit_elems", ctypes.c_int), ("unit_order", ctypes.c_int)]


class TriotError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__("%s: %s (%s)" % (what or "triot", name, status_string(status)))
        self.status = status


_lib = None

NOALLOC_SCRATCH_BYTES = 8 << 20

EXPORTS = ["triot_apply", "triot_apply_noalloc", "triot_workspace_size", "triot_batch_create", "triot_batch_destroy",
           "triot_apply_batched", "triot_batch_launch", "triot_batch_info", "triot_batch_set_schedule",
           "triot_batch_get_schedule", "triot_batch_autotune",
           "triot_autotune", "triot_tune_reset", "triot_schedule_set", "triot_schedule_get",
           "triot_status_string", "triot_divmod_magic", "triot_plan_describe"]


def lib():
    """The loaded library (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libtriot.so is not built (%s); run `python -m paper_1608_00099_amd.build`"
                           % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    pI64 = ctypes.POINTER(ctypes.c_int64)
    pP = ctypes.POINTER(ctypes.c_void_p)
    L.triot_apply.restype = I
    L.triot_apply.argtypes = [I, I, I, pI64, pI64, pP, pI64, P, P, P, SZ, P]
    L.triot_apply_noalloc.restype = I
    L.triot_apply_noalloc.argtypes = [I, I, I, pI64, pI64, pP, pI64, P, P, P]
    L.triot_workspace_size.restype = SZ
    L.triot_workspace_size.argtypes = [I, I, I, pI64, pI64]
    L.triot_batch_create.restype = I
    L.triot_batch_create.argtypes = [ctypes.POINTER(P)]
    L.triot_batch_destroy.restype = None
    L.triot_batch_destroy.argtypes = [P]
    L.triot_apply_batched.restype = I
    L.triot_apply_batched.argtypes = [I, I, ctypes.POINTER(Item), P, P, P]
    L.triot_batch_launch.restype = I
    L.triot_batch_launch.argtypes = [P, P]
    L.triot_batch_info.restype = I
    L.triot_batch_info.argtypes = [P, pI64, ctypes.POINTER(I), ctypes.POINTER(I)]
    L.triot_batch_set_schedule.restype = I
    L.triot_batch_set_schedule.argtypes = [P, ctypes.POINTER(Schedule)]
    L.triot_batch_get_schedule.restype = I
    L.triot_batch_get_schedule.argtypes = [P, ctypes.POINTER(Schedule)]
    L.triot_batch_autotune.restype = I
    L.triot_batch_autotune.argtypes = [P, I, I, ctypes.POINTER(Item), P, P, ctypes.c_char_p]
    L.triot_autotune.restype = I
    L.triot_autotune.argtypes = [I, I, I, pI64, pI64, pP, pI64, P, P, P, SZ, P, ctypes.c_char_p]
    L.triot_tune_reset.restype = None
    L.triot_tune_reset.argtypes = []
    L.triot_schedule_set.restype = I
    L.triot_schedule_set.argtypes = [I, I, I, pI64, pI64, pP, pI64, P, ctypes.POINTER(Schedule)]
    L.triot_schedule_get.restype = I
    L.triot_schedule_get.argtypes = [I, I, I, pI64, pI64, pP, pI64, P, ctypes.POINTER(Schedule)]
    L.triot_status_string.restype = ctypes.c_char_p
    L.triot_status_string.argtypes = [I]
    L.triot_divmod_magic.restype = I
    L.triot_divmod_magic.argtypes = [ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                     ctypes.POINTER(ctypes.c_uint32)]
    L.triot_plan_describe.restype = I
    L.triot_plan_describe.argtypes = [I, I, I, pI64, pI64, pP, pI64, P, ctypes.POINTER(PlanInfo)]
    _lib = L
    return L


def _i64_array(vals):
    if vals is None:
        return None
    vals = [int(v) for v in vals]
    return (ctypes.c_int64 * max(len(vals), 1))(*vals) if vals else (ctypes.c_int64 * 1)(0)


def _ptr_array(ptrs):
    return (ctypes.c_void_p * max(len(ptrs), 1))(*[ctypes.c_void_p(int(p) if p else 0) for p in ptrs])


def _params_ptr(params):
    if params is None:
        return None
    return ctypes.cast(ctypes.pointer(params), ctypes.c_void_p)


def status_string(status: int) -> str:
    return lib().triot_status_string(int(status)).decode()


def triot_apply(op, n_tensors, d, shapes, counter_shape, tensors, bases, params, out,
                workspace, workspace_bytes, stream) -> int:
    """Marshal and call triot_apply; returns the triot_status."""
    shapes_a = _i64_array([v for s in shapes for v in s] if d else [])
    counter_a = _i64_array(counter_shape) if counter_shape is not None else None
    bases_a = _i64_array(bases) if bases is not None else None
    return lib().triot_apply(int(op), int(n_tensors), int(d), shapes_a,
                             counter_a, _ptr_array(tensors), bases_a,
                             _params_ptr(params), ctypes.c_void_p(int(out) if out else 0),
                             ctypes.c_void_p(int(workspace) if workspace else 0),
                             int(workspace_bytes), ctypes.c_void_p(int(stream) if stream else 0))


def triot_apply_noalloc(op, n_tensors, d, shapes, counter_shape, tensors, bases, params,
                        out, stream) -> int:
    """Marshal and call triot_apply_noalloc; returns the triot_status."""
    shapes_a = _i64_array([v for s in shapes for v in s] if d else [])
    counter_a = _i64_array(counter_shape) if counter_shape is not None else None
    bases_a = _i64_array(bases) if bases is not None else None
    return lib().triot_apply_noalloc(int(op), int(n_tensors), int(d), shapes_a, counter_a,
                                     _ptr_array(tensors), bases_a, _params_ptr(params),
                                     ctypes.c_void_p(int(out) if out else 0),
                                     ctypes.c_void_p(int(stream) if stream else 0))


def triot_workspace_size(op, n_tensors, d, shapes, counter_shape=None) -> int:
    shapes_a = _i64_array([v for s in shapes for v in s] if d else [])
    counter_a = _i64_array(counter_shape) if counter_shape is not None else None
    return int(lib().triot_workspace_size(int(op), int(n_tensors), int(d), shapes_a, counter_a))


def triot_plan_describe(op, n_tensors, d, shapes, counter_shape, tensors, bases=None, params=None):
    info = PlanInfo()
    shapes_a = _i64_array([v for s in shapes for v in s] if d else [])
    counter_a = _i64_array(counter_shape) if counter_shape is not None else None
    bases_a = _i64_array(bases) if bases is not None else None
    st = lib().triot_plan_describe(int(op), int(n_tensors), int(d), shapes_a, counter_a,
                                   _ptr_array(tensors), bases_a, _params_ptr(params),
                                   ctypes.byref(info))
    return st, info


def triot_divmod_magic(c: int):
    m = ctypes.c_uint32()
    s = ctypes.c_uint32()
    st = lib().triot_divmod_magic(ctypes.c_uint32(c), ctypes.byref(m), ctypes.byref(s))
    return st, m.value, s.value


def triot_autotune(op, n_tensors, d, shapes, counter_shape, tensors, bases, params, out,
                   workspace, workspace_bytes, stream, cache_path=None) -> int:
    shapes_a = _i64_array([v for s in shapes for v in s] if d else [])
    counter_a = _i64_array(counter_shape) if counter_shape is not None else None
    bases_a = _i64_array(bases) if bases is not None else None
    return lib().triot_autotune(int(op), int(n_tensors), int(d), shapes_a, counter_a,
                                _ptr_array(tensors), bases_a, _params_ptr(params),
                                ctypes.c_void_p(int(out) if out else 0),
                                ctypes.c_void_p(int(workspace) if workspace else 0),
                                int(workspace_bytes), ctypes.c_void_p(int(stream) if stream else 0),
                                cache_path.encode() if cache_path else None)


def triot_tune_reset() -> None:
    lib().triot_tune_reset()


def triot_schedule_set(op, n_tensors, d, shapes, counter_shape, tensors, bases, params,
                       schedule) -> int:
    shapes_a = _i64_array([v for s in shapes for v in s] if d else [])
    counter_a = _i64_array(counter_shape) if counter_shape is not None else None
    bases_a = _i64_array(bases) if bases is not None else None
    return lib().triot_schedule_set(int(op), int(n_tensors), int(d), shapes_a, counter_a,
                                    _ptr_array(tensors), bases_a, _params_ptr(params),
                                    ctypes.byref(schedule))


def triot_schedule_get(op, n_tensors, d, shapes, counter_shape, tensors, bases, params):
    shapes_a = _i64_array([v for s in shapes for v in s] if d else [])
    counter_a = _i64_array(counter_shape) if counter_shape is not None else None
    bases_a = _i64_array(bases) if bases is not None else None
    sch = Schedule()
    st = lib().triot_schedule_get(int(op), int(n_tensors), int(d), shapes_a, counter_a,
                                  _ptr_array(tensors), bases_a, _params_ptr(params),
                                  ctypes.byref(sch))
    return st, sch


def triot_batch_create():
    h = ctypes.c_void_p()
    st = lib().triot_batch_create(ctypes.byref(h))
    return st, h


def triot_batch_destroy(handle) -> None:
    lib().triot_batch_destroy(handle)


def triot_batch_set_schedule(handle, schedule) -> int:
    return lib().triot_batch_set_schedule(handle, ctypes.byref(schedule))


def triot_batch_get_schedule(handle):
    sch = Schedule()
    st = lib().triot_batch_get_schedule(handle, ctypes.byref(sch))
    return st, sch


def _items_array(items):
    """Marshal [(d, n_tensors, shapes, counter_shape or None, ptrs, bases or
    None)] into a triot_item array; returns it with the arrays it points to."""
    keep = []
    arr = (Item * max(len(items), 1))()
    for i, (d, n, shapes, counter, ptrs, bases) in enumerate(items):
        sh = _i64_array([v for s in shapes for v in s] if d else [])
        ct = _i64_array(counter) if counter is not None else None
        pt = _ptr_array(ptrs)
        bs = _i64_array(bases) if bases is not None else None
        keep.append((sh, ct, pt, bs))
        arr[i].d = int(d)
        arr[i].n_tensors = int(n)
        arr[i].shapes = ctypes.cast(sh, ctypes.POINTER(ctypes.c_int64))
        arr[i].counter_shape = ctypes.cast(ct, ctypes.POINTER(ctypes.c_int64)) if ct is not None else None
        arr[i].tensors = ctypes.cast(pt, ctypes.POINTER(ctypes.c_void_p))
        arr[i].bases = ctypes.cast(bs, ctypes.POINTER(ctypes.c_int64)) if bs is not None else None
    return arr, keep


def triot_batch_autotune(handle, op, items, params, stream, cache_path=None) -> int:
    """items as for triot_apply_batched."""
    arr, keep = _items_array(items)
    st = lib().triot_batch_autotune(handle, int(op), len(items), arr, _params_ptr(params),
                                    ctypes.c_void_p(int(stream) if stream else 0),
                                    cache_path.encode() if cache_path else None)
    del keep
    return st


def triot_apply_batched(op, items, params, handle, stream) -> int:
    """items: list of (d, n_tensors, shapes, counter_shape or None, ptrs, bases or None).
    The marshalled arrays live until the call returns (the library copies
    what it keeps)."""
    arr, keep = _items_array(items)
    st = lib().triot_apply_batched(int(op), len(items), arr, _params_ptr(params), handle,
                                   ctypes.c_void_p(int(stream) if stream else 0))
    del keep
    return st


def triot_batch_launch(handle, stream) -> int:
    return lib().triot_batch_launch(handle, ctypes.c_void_p(int(stream) if stream else 0))


def triot_batch_info(handle):
    u = ctypes.c_int64()
    b = ctypes.c_int()
    r = ctypes.c_int()
    st = lib().triot_batch_info(handle, ctypes.byref(u), ctypes.byref(b), ctypes.byref(r))
    return st, u.value, b.value, r.value
