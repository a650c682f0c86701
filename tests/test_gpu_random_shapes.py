"""Seeded random layouts for the reductions (inner product, marginals,
bounding box, moments) against the CPU oracle: dimensions 1..6, extents
1..40 with many multiples of 4 (the 16-byte and staged paths), one to three
operands whose shapes are the counter or larger (windows), and random keep
masks.  Integer-valued weights make every float64 sum exact whatever the
order, so the inner product and marginals are compared bit for bit; the
moments within the float32 bound of the other moments tests."""
import numpy as np
import pytest

import oracle
from paper_1608_00099_amd import api, inputs
from tests.gpu_util import announce, dev, host

pytestmark = pytest.mark.gpu

N_CASES = 120


def _case(seed):
    g = inputs.rng(7, 100, seed)
    d = int(g.integers(1, 7))
    choices = [1, 2, 3, 4, 5, 7, 8, 12, 16, 20, 32, 40]
    while True:                               # at most 2^20 points
        counter = tuple(int(g.choice(choices)) for _ in range(d))
        if int(np.prod(counter)) <= 1 << 20:
            break
    n = int(g.integers(1, 4))
    shapes = []
    for k in range(n):
        if k == 0 or g.random() < 0.5:
            shapes.append(counter)            # the counter itself: contiguous
        else:
            shapes.append(tuple(c + int(g.integers(0, 5)) for c in counter))
    keep = tuple(int(g.integers(0, 2)) for _ in range(d))
    vals = [g.integers(-3, 4, size=s).astype(np.float32) for s in shapes]
    return counter, shapes, keep, vals


@pytest.mark.parametrize("seed", range(N_CASES))
def test_random_layouts(seed):
    counter, shapes, keep, vals = _case(seed)
    announce("random layouts", seed, counter, shapes, keep)
    # shapes larger than the counter are windows at base 0: the library
    # takes the intersection of the operands as the counter
    inter = tuple(min(s[i] for s in shapes) for i in range(len(counter)))
    assert inter == counter
    g = [dev(v) for v in vals]
    if len(vals) >= 2:
        want = oracle.dot(counter, vals, shapes)
        o32, o64 = api.dot(*g)
        assert host(o64)[0] == want, (host(o64)[0], want)
    want = oracle.marginal(counter, keep, vals, shapes)
    o32, o64 = api.marginal(g[0], keep, others=g[1:])
    assert np.array_equal(host(o64), want)
    want = oracle.bbox(counter, vals, shapes)
    got = host(api.bbox(*g))
    assert np.array_equal(got, want), (got, want)
    # moments of nonnegative weights (a PMF up to normalisation)
    pos = [np.abs(v) + 1.0 for v in vals]
    cov = len(counter) <= 8
    want = oracle.moments(counter, [p.reshape(-1) for p in pos], shapes, cov=cov)
    o32, o64 = api.moments(dev(pos[0]), cov=cov, others=[dev(p) for p in pos[1:]])
    got = host(o64)
    nmom = len(want)
    # the GPU's sums are exact here (integer weights, half-integer centred
    # coordinates); the oracle's second pass rounds its centred products,
    # about 1e-13 of the largest moment, which a covariance near zero shows
    # as a large relative error: judge every moment against that scale
    big = float(np.max(np.abs(want[1:]))) if nmom > 1 else 0.0
    scale = np.maximum(np.abs(want), big)
    assert np.all(np.abs(got[:nmom] - want) <= 1e-9 * scale), (got[:nmom], want)
