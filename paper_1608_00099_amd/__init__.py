"""MI355X-native co-iteration over tensors of run-time dimension and shape.

A from-scratch gfx950 implementation of the hot path of Heyl & Serang,
"TRIOT: Faster tensor manipulation in C++11" (arXiv 1608.00099): flat ->
tuple decode by magic-number division, row-major (Horner) offsets in every
operand, and the operations that co-iterate over them -- zero-pad
embedding and crop, element-wise products over shared tuples,
index-weighted moments -- with batched (one persistent hipGraph launch) and
differentiable (hand-written adjoint kernels) forms.

The kernels live in libtriot.so behind the C ABI of include/triot.h;
``_lib`` binds it with ctypes, ``api`` adds torch-tensor helpers and
``autograd`` the differentiable Functions.  Submodules load lazily so that
``inputs`` (seeded workload generators) imports without the library.
"""
import importlib

__all__ = ["api", "autograd", "inputs", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module("." + name, __name__)
    raise AttributeError(name)
