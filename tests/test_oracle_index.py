"""Pins for the oracle's index arithmetic (Section 1 of the paper).

Every check compares the oracle against something other than itself: the
worked example printed in the paper, hand-derived values, numpy's
``ravel_multi_index`` / ``unravel_index``, ``itertools.product`` and
hard-coded nested loops (the paper's Algorithm 1 style), and two
independent re-indexing computations written here (remainder/quotient and
shift/mask for power-of-two shapes).
"""
import itertools
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.txt")


def _golden_rows():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        t, s, f = [p.strip() for p in line.split(";")]
        rows.append((tuple(int(v) for v in t.split(",")),
                     tuple(int(v) for v in s.split(",")), int(f)))
    return rows


def test_worked_example_651():
    rows = _golden_rows()
    assert rows, "golden fixture is empty"
    for t, s, f in rows:
        assert oracle.flat_index(t, s) == f
        assert oracle.unflatten(f, s) == t


def test_hand_derived_examples():
    # The worked example's tuple in a power-of-two shape:
    # ((2*16 + 0)*8 + 4)*8 + 1 = 2081.
    assert oracle.flat_index((2, 0, 4, 1), (8, 16, 8, 8)) == 2081
    # The last element of a shape sits at prod(shape) - 1.
    assert oracle.flat_index((3, 8, 6, 4), (4, 9, 7, 5)) == 4 * 9 * 7 * 5 - 1
    # 1-d: the index is the tuple itself.
    assert oracle.flat_index((17,), (40,)) == 17
    # d = 0: the single (empty) tuple sits at offset 0.
    assert oracle.flat_index((), ()) == 0


@pytest.mark.parametrize("seed", range(6))
def test_flat_index_matches_numpy(seed):
    rng = np.random.default_rng(100 + seed)
    d = int(rng.integers(1, 9))
    shape = tuple(int(v) for v in rng.integers(1, 40, size=d))
    for _ in range(50):
        t = tuple(int(rng.integers(0, s)) for s in shape)
        assert oracle.flat_index(t, shape) == int(np.ravel_multi_index(t, shape))
        f = int(rng.integers(0, int(np.prod(shape))))
        assert oracle.unflatten(f, shape) == tuple(int(v) for v in np.unravel_index(f, shape))


def test_large_shape_uses_64bit():
    shape = (3000, 3000, 3000)          # 2.7e10 elements > 2^32
    t = (2999, 2998, 2997)
    assert oracle.flat_index(t, shape) == int(np.ravel_multi_index(t, shape))


@pytest.mark.parametrize("counter", [(3,), (2, 3), (3, 1, 4), (2, 3, 2, 2), (1, 1), (5, 1, 1, 2)])
def test_traversal_is_lexicographic(counter):
    got = oracle.tuples(counter)
    assert got == list(itertools.product(*[range(c) for c in counter]))


def _nested_loops(counter):
    """Hard-coded loop nests for d <= 4 (one loop per axis, outermost
    first), as the paper's Algorithm 1 writes them."""
    d = len(counter)
    out = []
    if d == 1:
        for i0 in range(counter[0]):
            out.append((i0,))
    elif d == 2:
        for i0 in range(counter[0]):
            for i1 in range(counter[1]):
                out.append((i0, i1))
    elif d == 3:
        for i0 in range(counter[0]):
            for i1 in range(counter[1]):
                for i2 in range(counter[2]):
                    out.append((i0, i1, i2))
    elif d == 4:
        for i0 in range(counter[0]):
            for i1 in range(counter[1]):
                for i2 in range(counter[2]):
                    for i3 in range(counter[3]):
                        out.append((i0, i1, i2, i3))
    return out


def _nested_loop_offsets(counter, shape):
    """The inline Horner index of Algorithm 1, written per depth."""
    d = len(counter)
    offs = []
    for t in _nested_loops(counter):
        if d == 1:
            offs.append(t[0])
        elif d == 2:
            offs.append(t[0] * shape[1] + t[1])
        elif d == 3:
            offs.append((t[0] * shape[1] + t[1]) * shape[2] + t[2])
        else:
            offs.append(((t[0] * shape[1] + t[1]) * shape[2] + t[2]) * shape[3] + t[3])
    return offs


@pytest.mark.parametrize("counter,shape", [
    ((7,), (9,)), ((3, 4), (5, 6)), ((2, 3, 4), (4, 5, 6)), ((2, 3, 2, 3), (3, 3, 5, 4)),
    ((4, 9, 7, 5), (4, 9, 7, 5))])
def test_traversal_and_offsets_match_nested_loops(counter, shape):
    assert oracle.tuples(counter) == _nested_loops(counter)
    got = oracle.index(counter, [shape])[0].tolist()
    assert got == _nested_loop_offsets(counter, shape)


def test_own_shape_traversal_visits_offsets_in_order():
    shape = (3, 5, 2, 4)
    offs = oracle.index(shape, [shape])[0]
    assert offs.tolist() == list(range(int(np.prod(shape))))


def test_extent_zero_and_scalar():
    assert oracle.tuples((3, 0, 2)) == []
    assert oracle.tuples(()) == [()]
    assert oracle.index((), [(), ()], bases=[5, 7]).tolist() == [[5], [7]]


def _reindex_divmod(f, shape, new_shape):
    """Flat index in ``shape`` -> flat index in ``new_shape`` by peeling
    digits with remainder/quotient, last axis first (Section 1)."""
    new_f, weight = 0, 1
    for i in range(len(shape) - 1, -1, -1):
        digit = f % shape[i]
        f //= shape[i]
        new_f += digit * weight
        weight *= new_shape[i]
    return new_f


def _reindex_pow2(f, log_shape, new_log_shape):
    """The same for power-of-two extents, with masks and shifts."""
    new_f, shift = 0, 0
    for i in range(len(log_shape) - 1, -1, -1):
        digit = f & ((1 << log_shape[i]) - 1)
        f >>= log_shape[i]
        new_f |= digit << shift
        shift += new_log_shape[i]
    return new_f


def test_reindex_cross_checks():
    shape, big = (9, 4, 6), (12, 7, 10)
    offs = oracle.index(shape, [shape, big])
    for f in range(int(np.prod(shape))):
        assert offs[1, f] == _reindex_divmod(f, shape, big)
    lg, lgb = (3, 2, 4), (4, 3, 5)
    sh = tuple(1 << v for v in lg)
    shb = tuple(1 << v for v in lgb)
    offs = oracle.index(sh, [sh, shb])
    for f in range(int(np.prod(sh))):
        assert offs[1, f] == _reindex_pow2(f, lg, lgb)


def test_index_with_bases_matches_numpy_windows():
    rng = np.random.default_rng(7)
    parent = (6, 7, 8)
    counter = (3, 4, 5)
    start = (2, 1, 3)
    base = int(np.ravel_multi_index(start, parent))
    offs = oracle.index(counter, [parent, counter], bases=[base, 0])
    idx = np.arange(int(np.prod(parent))).reshape(parent)
    want = idx[2:5, 1:5, 3:8].reshape(-1)
    assert offs[0].tolist() == want.tolist()
    assert offs[1].tolist() == list(range(int(np.prod(counter))))
    # A window that runs past the parent is rejected (one check per call).
    with pytest.raises(oracle.OracleError) as e:
        oracle.index(counter, [parent], bases=[int(np.ravel_multi_index((4, 0, 0), parent))])
    assert e.value.code == oracle.EBOUNDS
    del rng
