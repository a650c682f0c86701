"""CPU oracle for co-iteration (TEST INFRASTRUCTURE ONLY).

A plain, slow, obviously-correct reference for the operations of Heyl &
Serang, "TRIOT: Faster tensor manipulation in C++11" (arXiv 1608.00099):
zero-pad embedding / crop copies, element-wise products over shared
tuples, index-weighted moments (Algorithm 11) and their adjoints, the
inner product and update of benchmarks 2 and 3, marginalization, the
nonzero bounding box and the naive convolution (Algorithms 14 and 15).  The
arithmetic lives in ``triot_oracle.c`` (built with gcc, contraction off);
this module only marshals numpy arrays.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU
baseline may import this package.  The product library never does, and
this package imports nothing from it.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against the paper's worked example, hard-coded nested loops, numpy
library routines, closed forms, exact rational brute force and finite
differences.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "triot_oracle.c")
_LIB = os.path.join(_HERE, "libtriot_oracle.so")
_lib = None

OK, EINVAL, EDIM, EBOUNDS = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain ISO C, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
            "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _configure(lib):
    """Declare argument types on a loaded oracle library."""
    P = ctypes.c_void_p
    I = ctypes.c_int
    L = ctypes.c_int64
    lib.oracle_flat_index.restype = ctypes.c_uint64
    lib.oracle_flat_index.argtypes = [P, P, I]
    lib.oracle_next_tuple.restype = I
    lib.oracle_next_tuple.argtypes = [P, P, I]
    lib.oracle_unflatten.restype = None
    lib.oracle_unflatten.argtypes = [ctypes.c_uint64, P, I, P]
    lib.oracle_copy.argtypes = [I, P, P, P, L, P, P, L, I]
    lib.oracle_embed_fill.argtypes = [I, P, P, P, L, P, P, L, I]
    lib.oracle_mul_acc.argtypes = [I, P, P, P, L, P, P, L, P, P, L, I]
    lib.oracle_mul.argtypes = [I, P, P, P, L, P, P, L, P, P, L, I]
    lib.oracle_index.argtypes = [I, I, P, P, P, P]
    lib.oracle_moments.argtypes = [I, I, P, P, P, P, I, I, P]
    lib.oracle_moments_adj.argtypes = [I, P, P, P, L, I, P, P, I]
    lib.oracle_mul_adj.argtypes = [I, P, P, P, P, P, P, P, P, I]
    lib.oracle_dot.argtypes = [I, I, P, P, P, P, I, P]
    lib.oracle_xpyx_mz.argtypes = [I, P, P, P, L, P, P, L, P, P, L, I]
    lib.oracle_marginal.argtypes = [I, I, P, P, P, P, P, I, P]
    lib.oracle_bbox.argtypes = [I, I, P, P, P, P, I, P]
    lib.oracle_conv.argtypes = [I, P, P, P, P, P]
    return lib


def _load():
    global _lib
    if _lib is None:
        # ORACLE_LIB names a deliberately broken build of this same source,
        # used only by the mutation test that checks the pins catch it.
        path = os.environ.get("ORACLE_LIB") or build()
        _lib = _configure(ctypes.CDLL(path))
    return _lib


def _i64(seq):
    a = np.ascontiguousarray(np.asarray(list(seq), dtype=np.int64))
    return a


def _u64(seq):
    return np.ascontiguousarray(np.asarray(list(seq), dtype=np.uint64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _flat(a: np.ndarray) -> np.ndarray:
    if not a.flags.c_contiguous:
        raise ValueError("oracle operands must be C-contiguous buffers")
    return a


def _check(rc: int, what: str):
    if rc != OK:
        raise OracleError(rc, what)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed with oracle code %d" % (what, code))
        self.code = code


# ---------------------------------------------------------------------------
# Index arithmetic
# ---------------------------------------------------------------------------

def flat_index(t, shape) -> int:
    """Row-major flat index of tuple ``t`` in ``shape`` (Section 1)."""
    lib = _load()
    tt, ss = _u64(t), _u64(shape)
    return int(lib.oracle_flat_index(_ptr(tt), _ptr(ss), len(shape)))


def unflatten(f: int, shape):
    """Tuple of flat index ``f`` in ``shape`` by remainder/quotient."""
    lib = _load()
    ss = _u64(shape)
    out = np.zeros(max(len(shape), 1), dtype=np.uint64)
    lib.oracle_unflatten(ctypes.c_uint64(f), _ptr(ss), len(shape), _ptr(out))
    return tuple(int(v) for v in out[: len(shape)])


def tuples(counter):
    """All tuples of ``counter`` in the oracle's visiting order
    (increment-with-carry; Section 1)."""
    lib = _load()
    d = len(counter)
    c = _u64(counter)
    if any(v == 0 for v in counter):
        return []
    t = np.zeros(max(d, 1), dtype=np.uint64)
    out = []
    while True:
        out.append(tuple(int(v) for v in t[:d]))
        if not lib.oracle_next_tuple(_ptr(t), _ptr(c), d):
            break
    return out


# ---------------------------------------------------------------------------
# Operations on numpy buffers.  Every operand is (buffer, shape, base): a
# C-contiguous parent buffer viewed with the parent's row-major ``shape``;
# ``base`` is the element offset of the window start (Section 4, slices).
# ---------------------------------------------------------------------------

def copy(counter, dst, dst_shape, src, src_shape, dst_base=0, src_base=0):
    lib = _load()
    assert dst.dtype.itemsize == src.dtype.itemsize
    rc = lib.oracle_copy(len(counter), _ptr(_i64(counter)), _ptr(_flat(dst)),
                         _ptr(_i64(dst_shape)), dst_base, _ptr(_flat(src)),
                         _ptr(_i64(src_shape)), src_base, dst.dtype.itemsize)
    _check(rc, "copy")
    return dst


def embed_fill(counter, dst, dst_shape, src, src_shape, dst_base=0, src_base=0):
    lib = _load()
    assert dst.dtype.itemsize == src.dtype.itemsize
    rc = lib.oracle_embed_fill(len(counter), _ptr(_i64(counter)), _ptr(_flat(dst)),
                               _ptr(_i64(dst_shape)), dst_base, _ptr(_flat(src)),
                               _ptr(_i64(src_shape)), src_base, dst.dtype.itemsize)
    _check(rc, "embed_fill")
    return dst


def _fdt(*arrs):
    dt = arrs[0].dtype
    assert all(a.dtype == dt for a in arrs), "operands must share a dtype"
    assert dt in (np.float32, np.float64)
    return 1 if dt == np.float64 else 0


def mul_acc(counter, x, xs, y, ys, z, zs, xb=0, yb=0, zb=0):
    lib = _load()
    f64 = _fdt(x, y, z)
    rc = lib.oracle_mul_acc(len(counter), _ptr(_i64(counter)),
                            _ptr(_flat(x)), _ptr(_i64(xs)), xb,
                            _ptr(_flat(y)), _ptr(_i64(ys)), yb,
                            _ptr(_flat(z)), _ptr(_i64(zs)), zb, f64)
    _check(rc, "mul_acc")
    return x


def mul(counter, out, os_, a, as_, b, bs, ob=0, ab=0, bb=0):
    lib = _load()
    f64 = _fdt(out, a, b)
    rc = lib.oracle_mul(len(counter), _ptr(_i64(counter)),
                        _ptr(_flat(out)), _ptr(_i64(os_)), ob,
                        _ptr(_flat(a)), _ptr(_i64(as_)), ab,
                        _ptr(_flat(b)), _ptr(_i64(bs)), bb, f64)
    _check(rc, "mul")
    return out


def index(counter, shapes, bases=None) -> np.ndarray:
    """Offsets of every counter tuple in every operand: int64 [n, N]."""
    lib = _load()
    n, d = len(shapes), len(counter)
    N = int(np.prod(counter, dtype=np.int64)) if d else 1
    out = np.zeros((n, max(N, 0)), dtype=np.int64)
    sh = _i64([v for s in shapes for v in s]) if d else np.zeros(1, np.int64)
    bs = _i64(bases if bases is not None else [0] * n)
    rc = lib.oracle_index(n, d, _ptr(_i64(counter) if d else np.zeros(1, np.int64)),
                          _ptr(sh), _ptr(bs), _ptr(out))
    _check(rc, "index")
    return out


def moments(counter, tensors, shapes, bases=None, cov=True) -> np.ndarray:
    """[M, E_0..E_{d-1}, upper-triangle C] in float64 (Algorithm 11)."""
    lib = _load()
    n, d = len(tensors), len(counter)
    f64 = _fdt(*tensors)
    nout = 1 + d + d * (d + 1) // 2
    out = np.zeros(nout, dtype=np.float64)
    ptrs = (ctypes.c_void_p * n)(*[_flat(t).ctypes.data for t in tensors])
    sh = _i64([v for s in shapes for v in s]) if d else np.zeros(1, np.int64)
    bs = _i64(bases if bases is not None else [0] * n)
    rc = lib.oracle_moments(n, d, _ptr(_i64(counter) if d else np.zeros(1, np.int64)),
                            ptrs, _ptr(sh), _ptr(bs), f64, 2 if cov else 1, _ptr(out))
    _check(rc, "moments")
    if not cov:
        out[1 + d:] = 0.0
    return out


def moments_adj(counter, g, g_shape, mom, gmom, cov=True, g_base=0):
    lib = _load()
    f64 = 1 if g.dtype == np.float64 else 0
    m = np.ascontiguousarray(mom, dtype=np.float64)
    gm = np.ascontiguousarray(gmom, dtype=np.float64)
    d = len(counter)
    rc = lib.oracle_moments_adj(d, _ptr(_i64(counter) if d else np.zeros(1, np.int64)),
                                _ptr(_flat(g)), _ptr(_i64(g_shape) if d else np.zeros(1, np.int64)),
                                g_base, f64, _ptr(m), _ptr(gm), 2 if cov else 1)
    _check(rc, "moments_adj")
    return g


def mul_adj(ga, sa, gb, sb, gout, si, a, b):
    lib = _load()
    f64 = _fdt(ga, gb, gout, a, b)
    d = len(sa)
    rc = lib.oracle_mul_adj(d, _ptr(_flat(ga)), _ptr(_i64(sa)), _ptr(_flat(gb)),
                            _ptr(_i64(sb)), _ptr(_flat(gout)), _ptr(_i64(si)),
                            _ptr(_flat(a)), _ptr(_flat(b)), f64)
    _check(rc, "mul_adj")
    return ga, gb


def _operands(counter, tensors, shapes, bases):
    n, d = len(tensors), len(counter)
    ptrs = (ctypes.c_void_p * n)(*[_flat(t).ctypes.data for t in tensors])
    sh = _i64([v for s in shapes for v in s]) if d else np.zeros(1, np.int64)
    bs = _i64(bases if bases is not None else [0] * n)
    cc = _i64(counter) if d else np.zeros(1, np.int64)
    return n, d, ptrs, sh, bs, cc


def dot(counter, tensors, shapes, bases=None) -> float:
    """sum_t prod_k v_k(t) in float64 (benchmark 2's inner product)."""
    lib = _load()
    f64 = _fdt(*tensors)
    n, d, ptrs, sh, bs, cc = _operands(counter, tensors, shapes, bases)
    out = np.zeros(1, dtype=np.float64)
    rc = lib.oracle_dot(n, d, _ptr(cc), ptrs, _ptr(sh), _ptr(bs), f64, _ptr(out))
    _check(rc, "dot")
    return float(out[0])


def xpyx_mz(counter, x, xs, y, ys, z, zs, xb=0, yb=0, zb=0):
    """x[t] <- x[t] + y[t]*x[t] - z[t] (benchmark 3), three roundings."""
    lib = _load()
    f64 = _fdt(x, y, z)
    rc = lib.oracle_xpyx_mz(len(counter), _ptr(_i64(counter)),
                            _ptr(_flat(x)), _ptr(_i64(xs)), xb,
                            _ptr(_flat(y)), _ptr(_i64(ys)), yb,
                            _ptr(_flat(z)), _ptr(_i64(zs)), zb, f64)
    _check(rc, "xpyx_mz")
    return x


def marginal(counter, keep, tensors, shapes, bases=None) -> np.ndarray:
    """float64 sums of prod_k v_k(t) over the axes with keep[i] == 0; the
    result has the kept counter extents."""
    lib = _load()
    f64 = _fdt(*tensors)
    n, d, ptrs, sh, bs, cc = _operands(counter, tensors, shapes, bases)
    kshape = tuple(int(c) for c, k in zip(counter, keep) if k)
    out = np.zeros(max(int(np.prod(kshape, dtype=np.int64)), 1), dtype=np.float64)
    kk = np.ascontiguousarray(np.asarray([1 if k else 0 for k in keep] or [0], dtype=np.int32))
    rc = lib.oracle_marginal(n, d, _ptr(cc), _ptr(kk), ptrs, _ptr(sh), _ptr(bs), f64,
                             _ptr(out))
    _check(rc, "marginal")
    return out[: int(np.prod(kshape, dtype=np.int64))].reshape(kshape)


def bbox(counter, tensors, shapes, bases=None) -> np.ndarray:
    """int64 [d, 2]: per axis, min and max t_i where every operand is
    nonzero; all -1 when there is no such tuple."""
    lib = _load()
    f64 = _fdt(*tensors)
    n, d, ptrs, sh, bs, cc = _operands(counter, tensors, shapes, bases)
    out = np.zeros(max(2 * d, 1), dtype=np.int64)
    rc = lib.oracle_bbox(n, d, _ptr(cc), ptrs, _ptr(sh), _ptr(bs), f64, _ptr(out))
    _check(rc, "bbox")
    return out[: 2 * d].reshape(d, 2)


def conv(lhs, rhs) -> np.ndarray:
    """Naive convolution in Algorithm 14's loop order (float64)."""
    lib = _load()
    assert lhs.dtype == np.float64 and rhs.dtype == np.float64
    assert lhs.ndim == rhs.ndim
    d = lhs.ndim
    oshape = tuple(a + b - 1 for a, b in zip(lhs.shape, rhs.shape))
    out = np.zeros(max(int(np.prod(oshape, dtype=np.int64)), 1), dtype=np.float64)
    ls = _i64(lhs.shape) if d else np.zeros(1, np.int64)
    rs = _i64(rhs.shape) if d else np.zeros(1, np.int64)
    rc = lib.oracle_conv(d, _ptr(_flat(lhs)), _ptr(ls), _ptr(_flat(rhs)), _ptr(rs), _ptr(out))
    _check(rc, "conv")
    return out[: int(np.prod(oshape, dtype=np.int64))].reshape(oshape)
