"""FFT convolution end to end (pad with EMBED_FILL, rocFFT transforms,
crop with COPY) against the oracle's naive convolution (Algorithm 14).
The FFT's rounding differs from the naive sums: the float64 result must
lie within c * log2(N) * eps * (|lhs| conv |rhs|) of the oracle's, float32
within the same bound at float32's eps."""
import numpy as np
import pytest
import torch

import oracle
from paper_1608_00099_amd import fftconv, inputs
from tests.gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu


def _bound(l, r, eps):
    mag = oracle.conv(np.abs(l).astype(np.float64), np.abs(r).astype(np.float64))
    n = max(int(np.prod([fftconv.good_size(v) for v in mag.shape])), 2)
    return 16 * np.log2(n) * eps * mag.max()


@pytest.mark.parametrize("ls,rs", [((256, 8), (256, 8)), ((37,), (29,)), ((12, 9, 7), (5, 8, 6)),
                                   ((3, 4, 5, 6), (2, 3, 2, 3))])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_fft_conv_matches_naive_oracle(ls, rs, dt):
    announce("fft_conv", ls, rs, dt.__name__)
    rng = np.random.default_rng(400)
    l = rng.standard_normal(ls).astype(dt)
    r = rng.standard_normal(rs).astype(dt)
    want = oracle.conv(l.astype(np.float64), r.astype(np.float64))
    got = host(fftconv.fft_conv(dev(l), dev(r))).astype(np.float64)
    assert got.shape == want.shape
    assert np.max(np.abs(got - want)) <= _bound(l, r, np.finfo(dt).eps)


def test_fft_conv_batch_dims():
    announce("fft_conv batched dims")
    rng = np.random.default_rng(401)
    x = rng.standard_normal((5, 20, 11))
    y = rng.standard_normal((5, 7, 4))
    got = host(fftconv.fft_conv(dev(x), dev(y), batch_dims=1))
    for b in range(5):
        want = oracle.conv(np.ascontiguousarray(x[b]), np.ascontiguousarray(y[b]))
        assert np.max(np.abs(got[b] - want)) <= _bound(x[b], y[b], np.finfo(np.float64).eps)


def test_ragged_fft_conv_cfg4_like():
    # ragged pairs of uneven dimension and shape, as in the batched pad
    # workload (few pairs: the FFT library compiles a kernel per new size)
    pairs = inputs.cfg4_shapes(n_pairs=8)
    announce("ragged fft_conv", len(pairs))
    rng = np.random.default_rng(402)
    xs = [rng.standard_normal(sx) for sx, sy in pairs]
    ys = [rng.standard_normal(sy) for sx, sy in pairs]
    rf = fftconv.RaggedFFTConv()
    try:
        for rep in range(2):                     # second call replays the captured batches
            outs = rf([dev(x) for x in xs], [dev(y) for y in ys])
            for x, y, o in zip(xs, ys, outs):
                want = oracle.conv(np.ascontiguousarray(x), np.ascontiguousarray(y))
                got = host(o)
                assert got.shape == want.shape
                assert np.max(np.abs(got - want)) <= _bound(x, y, np.finfo(np.float64).eps)
    finally:
        rf.close()
