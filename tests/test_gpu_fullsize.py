"""Full benchmark sizes, in the launch configuration the benchmark times,
compared with the oracle element by element.

  - The run-time-dimension sweep d = 2..8 with ~2^26-element tensors:
    pad-embed into a shape enlarged by 1..16 per axis, and x += y*z over
    the intersection of three shapes.  Each launch runs with the schedule
    the benchmark pins for it (tuned/sweep_d2-8_mi355x.json), so the box,
    split, unit and lane geometry checked here is the one that is timed.
  - Benchmark 1 of Section 3 at the paper's shape: the crop
    (2^10, 2^9, 2^8) -> (2^9, 2^9, 2^5) in float32 and float64, launched
    as the benchmark launches it (the library's default schedule).

Inputs are drawn on the host by the seeded recipes, copied to the device,
and the whole output (every element of the destination, including what
must stay untouched) is copied back and compared with the oracle's output
on the same host inputs, bit for bit."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1608_00099_amd import _lib as L
from paper_1608_00099_amd import api, inputs
from tests.gpu_util import announce, first_mismatch

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
with open(os.path.join(ROOT, "paper_1608_00099_amd", "tuned", "sweep_d2-8_mi355x.json")) as _f:
    SCHED = json.load(_f)


@pytest.fixture(autouse=True)
def _reset():
    yield
    api.tune_reset()
    torch.cuda.empty_cache()


def _prod(s):
    p = 1
    for v in s:
        p *= int(v)
    return p


def _to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(a).to("cuda")


def _same_bits(got: np.ndarray, want: np.ndarray, what):
    assert got.shape == want.shape and got.dtype == want.dtype
    if got.tobytes() != want.tobytes():
        raise AssertionError((what, "first mismatch (flat index, got, want, count)",
                              first_mismatch(got, want)))


@pytest.mark.parametrize("d", range(2, 9))
def test_pad_embed_full_size(d):
    src_s, dst_s = inputs.cfg2_pad_shapes(d)
    announce("full pad-embed vs oracle", d, src_s, dst_s)
    src = inputs.uniform(2, src_s, 50, d)
    want = np.zeros(_prod(dst_s), dtype=np.float32)
    oracle.copy(src_s, want, dst_s, src.reshape(-1), src_s)
    gsrc = _to_dev(src)
    gdst = torch.zeros(dst_s, dtype=torch.float32, device="cuda")
    api.schedule_set(L.OP_COPY, [gdst, gsrc], counter=src_s, params=L.CopyParams(4),
                     **SCHED["copy d=%d" % d])
    api.pad_embed_into(gdst, gsrc)
    got = gdst.cpu().numpy().reshape(-1)
    del gdst, gsrc
    _same_bits(got, want, ("pad-embed", d, src_s, dst_s))


@pytest.mark.parametrize("d", range(2, 9))
def test_mul_acc_full_size(d):
    xs, ys, zs = inputs.cfg2_inter_shapes(d)
    announce("full mul_acc vs oracle", d, xs, ys, zs)
    x = inputs.uniform(2, xs, 51, d)
    y = inputs.uniform(2, ys, 52, d)
    z = inputs.uniform(2, zs, 53, d)
    gx, gy, gz = _to_dev(x), _to_dev(y), _to_dev(z)
    want = x.reshape(-1).copy()
    oracle.mul_acc(xs, want, xs, y.reshape(-1), ys, z.reshape(-1), zs)
    api.schedule_set(L.OP_MUL_ACC, [gx, gy, gz], **SCHED["mul_acc d=%d" % d])
    api.mul_acc_(gx, gy, gz)
    got = gx.cpu().numpy().reshape(-1)
    _same_bits(got, want, ("mul_acc", d, xs, ys, zs))
    # the operands that are only read are unchanged
    _same_bits(gy.cpu().numpy(), y, ("mul_acc y changed", d))
    _same_bits(gz.cpu().numpy(), z, ("mul_acc z changed", d))
    del gx, gy, gz


B1_BIG = inputs.PAPER_B1_BIG
B1_SMALL = inputs.PAPER_B1_SMALL


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_benchmark1_crop_paper_shape(dtype):
    announce("benchmark 1 crop vs oracle", B1_BIG, "->", B1_SMALL, np.dtype(dtype).name)
    big = inputs.paper_b1_values(dtype)
    want = np.full(_prod(B1_SMALL), -1.0, dtype=dtype)   # the crop writes every element
    oracle.copy(B1_SMALL, want, B1_SMALL, big.reshape(-1), B1_BIG)
    gbig = _to_dev(big)
    gout = torch.full(B1_SMALL, -1.0, dtype=gbig.dtype, device="cuda")
    api.copy_(gout, gbig, counter=B1_SMALL)
    got = gout.cpu().numpy().reshape(-1)
    del gbig, gout
    _same_bits(got, want, ("benchmark-1 crop", np.dtype(dtype).name))
    # the oracle's crop is the leading block of the source (numpy slicing)
    assert np.array_equal(want.reshape(B1_SMALL), big[:512, :512, :32])
