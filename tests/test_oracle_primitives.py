"""Oracle primitives against things other than themselves.

Philox4x64-10 against numpy's independent implementation; the bounded draw and
the inverse-CDF pick against the uniformity they must provide (preimage sizes of
every outcome, found by bisection over the 64-bit word)."""
import numpy as np
import pytest

import oracle

M64 = (1 << 64) - 1


def numpy_block(counter: int, key):
    """numpy's Philox increments its 256-bit counter before producing a block, so
    block c of the oracle equals numpy's first block started from counter c-1."""
    c = (counter - 1) % (1 << 256)
    ctr = np.array([(c >> (64 * i)) & M64 for i in range(4)], dtype=np.uint64)
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=ctr)
    return bg.random_raw(4)


@pytest.mark.parametrize("counter", [0, 1, 2, 7, 2**32 + 5, 2**63 + 11, (5 << 64) | 9, (3 << 128) | 1])
@pytest.mark.parametrize("key", [(0, 0), (1, 0x4), (1, 0x51), (987654321, 0x52), (M64, M64)])
def test_philox_matches_numpy(counter, key):
    ctr = [(counter >> (64 * i)) & M64 for i in range(4)]
    got = oracle.philox(ctr, key)
    np.testing.assert_array_equal(got, numpy_block(counter, key))


def first_word_reaching(f, target):
    """Smallest 64-bit x with f(x) >= target (f monotone)."""
    lo, hi = 0, 1 << 64
    while lo < hi:
        mid = (lo + hi) // 2
        if f(mid) >= target:
            hi = mid
        else:
            lo = mid + 1
    return lo


@pytest.mark.parametrize("n", [1, 2, 3, 7, 10, 1000, 2**31 - 1, 2**40 + 3, 2**63 + 5, M64])
def test_bounded_draw_is_uniform(n):
    """Each outcome j in [0, n) must have floor(2^64/n) or ceil(2^64/n) preimages."""
    f = lambda x: oracle.bounded(x, n)
    assert f(0) == 0 and f(M64) == n - 1
    rng = np.random.Generator(np.random.PCG64(n % 1000))
    outs = sorted(set([0, 1, n - 1] + [int(x) for x in rng.integers(0, n, size=6, dtype=np.uint64)]))
    lo_size, hi_size = (1 << 64) // n, -((-(1 << 64)) // n)
    for j in outs:
        if j >= n:
            continue
        a = first_word_reaching(f, j)
        b = first_word_reaching(f, j + 1) if j + 1 < n else 1 << 64
        assert b - a in (lo_size, hi_size), (n, j, b - a)


def test_pick_inverse_cdf_measure():
    """Outcome i of pick() must own weight_i / total of the 64-bit word space (+-1),
    and zero-weight items must never be returned."""
    rng = np.random.Generator(np.random.PCG64(11))
    w = rng.integers(0, 50, size=40).astype(np.uint64)
    w[[0, 5, 6, 39]] = 0
    w[7] = 10**12
    acc = np.cumsum(w).astype(np.uint64)
    T = int(acc[-1])
    f = lambda x: oracle.pick(acc, x)
    bounds = [first_word_reaching(f, i) for i in range(len(w))] + [1 << 64]
    for i in range(len(w)):
        measure = bounds[i + 1] - bounds[i]
        ideal = int(w[i]) * (1 << 64) / T
        assert abs(measure - ideal) <= 1.0, (i, measure, ideal)
        if w[i] == 0:
            assert measure == 0
    xs = rng.integers(0, 2**63, size=2000, dtype=np.uint64) * 2 + 1
    for x in xs[:200]:
        assert w[f(int(x))] > 0
