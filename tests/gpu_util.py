"""Helpers shared by the GPU tests."""
import sys

import numpy as np
import torch


def announce(*what):
    """Name the case before any device work, so a failing run says which."""
    print("[case]", *what, flush=True)
    sys.stdout.flush()


def dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def bits_equal(a: np.ndarray, b: np.ndarray) -> bool:
    return a.dtype == b.dtype and a.shape == b.shape and a.tobytes() == b.tobytes()


def first_mismatch(a: np.ndarray, b: np.ndarray):
    fa = a.reshape(-1).view(np.uint8 if a.dtype.itemsize == 1 else
                            {4: np.uint32, 8: np.uint64}[a.dtype.itemsize])
    fb = b.reshape(-1).view(fa.dtype)
    idx = np.nonzero(fa != fb)[0]
    return (int(idx[0]), a.reshape(-1)[idx[0]], b.reshape(-1)[idx[0]], int(idx.size)) if idx.size else None


def rel_err(got, ref, floor=0.0):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.maximum(np.abs(ref), floor)
    with np.errstate(invalid="ignore", divide="ignore"):
        e = np.abs(got - ref) / den
    e[(got == ref)] = 0.0
    return e
