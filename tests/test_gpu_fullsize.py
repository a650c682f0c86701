"""Full benchmark sizes, in the launch configuration the benchmark times
(the sweep's pinned schedules, the file bench.py pins): the run-time-
dimension sweep d = 2..8 with ~2^26-element tensors.

At this size the oracle checks sampled points one by one (offsets from the
oracle's own index arithmetic, values gathered from the device), and whole
outputs are checked through properties that hold at any size: the embedded
block equals the source bit for bit and nothing outside it changed; x +=
y*z equals torch's separately rounded product-then-sum."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_1608_00099_amd import _lib as L
from paper_1608_00099_amd import api, inputs
from tests.gpu_util import announce

pytestmark = pytest.mark.gpu

NSAMPLE = 3000

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
with open(os.path.join(ROOT, "paper_1608_00099_amd", "tuned", "sweep_d2-8_mi355x.json")) as _f:
    SCHED = json.load(_f)


@pytest.fixture(autouse=True)
def _reset():
    yield
    api.tune_reset()


def _sl(counter):
    return tuple(slice(0, c) for c in counter)


def _sample_tuples(rng, counter, n):
    return [tuple(int(rng.integers(0, c)) for c in counter) for _ in range(n)]


def _bits(t):
    return t.contiguous().view(torch.int32)


@pytest.mark.parametrize("d", range(2, 9))
def test_pad_embed_full_size(d):
    src_s, dst_s = inputs.cfg2_pad_shapes(d)
    announce("full pad-embed", d, src_s, dst_s)
    dev = torch.device("cuda")
    src = inputs.uniform_torch(src_s, 5000 + d, dev)
    dst = torch.zeros(dst_s, dtype=torch.float32, device=dev)
    api.schedule_set(L.OP_COPY, [dst, src], counter=src_s, params=L.CopyParams(4),
                     **SCHED["copy d=%d" % d])
    api.pad_embed_into(dst, src)
    torch.cuda.synchronize()
    # the embedded block is the source, bit for bit
    assert torch.equal(_bits(dst[_sl(src_s)]), _bits(src))
    # and nothing else was written (the source is positive almost surely)
    assert int((dst != 0).sum()) == int((src != 0).sum())
    # sampled points through the oracle's own offsets
    rng = np.random.default_rng(d)
    ts = _sample_tuples(rng, src_s, NSAMPLE)
    od = torch.tensor([oracle.flat_index(t, dst_s) for t in ts], device=dev)
    os_ = torch.tensor([oracle.flat_index(t, src_s) for t in ts], device=dev)
    assert torch.equal(_bits(dst.reshape(-1)[od]), _bits(src.reshape(-1)[os_]))


@pytest.mark.parametrize("d", range(2, 9))
def test_mul_acc_full_size(d):
    xs, ys, zs = inputs.cfg2_inter_shapes(d)
    announce("full mul_acc", d, xs, ys, zs)
    dev = torch.device("cuda")
    x = inputs.uniform_torch(xs, 6000 + d, dev)
    y = inputs.uniform_torch(ys, 6100 + d, dev)
    z = inputs.uniform_torch(zs, 6200 + d, dev)
    x0 = x.clone()
    api.schedule_set(L.OP_MUL_ACC, [x, y, z], **SCHED["mul_acc d=%d" % d])
    api.mul_acc_(x, y, z)
    torch.cuda.synchronize()
    # torch reference: product, then sum, each rounded once
    prod = torch.mul(y[_sl(xs)], z[_sl(xs)])
    ref = torch.add(x0, prod)
    assert torch.equal(_bits(x), _bits(ref))
    del prod, ref
    # sampled points through the oracle's arithmetic and offsets
    rng = np.random.default_rng(100 + d)
    ts = _sample_tuples(rng, xs, 500)
    xo = torch.tensor([oracle.flat_index(t, xs) for t in ts], device=dev)
    yo = torch.tensor([oracle.flat_index(t, ys) for t in ts], device=dev)
    zo = torch.tensor([oracle.flat_index(t, zs) for t in ts], device=dev)
    xv = x0.reshape(-1)[xo].cpu().numpy()
    yv = y.reshape(-1)[yo].cpu().numpy()
    zv = z.reshape(-1)[zo].cpu().numpy()
    n = len(ts)
    oracle.mul_acc((n,), xv, (n,), yv, (n,), zv, (n,))
    got = x.reshape(-1)[xo].cpu().numpy()
    assert got.tobytes() == xv.tobytes()
