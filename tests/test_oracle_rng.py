"""Pins for the oracle's random streams (sample draw, Section 3 / Algorithm 3).

The oracle's Philox4x64-10 is written from the SC'11 definition; numpy's
Philox is an independent implementation of the same generator.  numpy
advances its 256-bit counter by one before producing a block, so block
``c`` of ours equals numpy's first block started at ``c - 1``.
"""
import numpy as np
import pytest
from scipy import stats


def _numpy_block(ctr, key):
    c = int(ctr[0]) | (int(ctr[1]) << 64) | (int(ctr[2]) << 128) | (int(ctr[3]) << 192)
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=words)
    return g.random_raw(4)


@pytest.mark.parametrize(
    "ctr,key",
    [
        ([0, 0, 0, 0], [0, 0]),
        ([1, 0, 0, 0], [0, 0]),
        ([0, 5, 0, 0], [7, 1]),  # borrow through word 0 in the numpy counter
        ([3, 11, 2, 0], [123456789, 2]),
        ([2**64 - 1, 2**64 - 1, 2**64 - 1, 2**64 - 1], [2**64 - 1, 2**64 - 1]),
        ([12345, 999, 77, 0], [0xDEADBEEF, 3]),
    ],
)
def test_philox_matches_numpy(orc, ctr, key):
    ours = orc.philox4x64_10(ctr, key)
    ref = _numpy_block(ctr, key)
    assert np.array_equal(ours, ref)


def test_sample_indices_are_mulhi_of_stream(orc):
    """idx_j = floor(r_j * m / 2^64) with r_j word j%4 of block j/4 of the
    stream key (seed, 0), counter (block, sample_id, 0, 0).  Recomputed with
    Python integers from numpy's Philox."""
    m, s, seed, sid = 1_000_003, 37, 99, 5
    idx = orc.draw_sample(m, s, seed, sid)
    ref = []
    for j in range(s):
        blk = _numpy_block([j // 4, sid, 0, 0], [seed, 0])
        ref.append((int(blk[j % 4]) * m) >> 64)
    assert idx.tolist() == ref


def test_sample_uniformity_chi2(orc):
    m, s = 1000, 1_000_000
    idx = orc.draw_sample(m, s, 2024, 0)
    assert idx.min() >= 0 and idx.max() < m
    counts = np.bincount(idx, minlength=m)
    chi2 = ((counts - s / m) ** 2 / (s / m)).sum()
    p = stats.chi2.sf(chi2, m - 1)
    assert p > 1e-6, (chi2, p)


def test_sample_streams_independent_of_each_other(orc):
    a = orc.draw_sample(10**9, 1000, 1, 0)
    b = orc.draw_sample(10**9, 1000, 1, 1)
    c = orc.draw_sample(10**9, 1000, 2, 0)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
    # deterministic
    assert np.array_equal(a, orc.draw_sample(10**9, 1000, 1, 0))
    # a prefix of a longer draw is the shorter draw
    assert np.array_equal(a[:333], orc.draw_sample(10**9, 333, 1, 0))


def test_scaling_study_generator_shapes():
    """Section 6.8: m = 3^(i+7) blob points in 10 dimensions plus 500 noise
    points in (-50, 50); s = min(5000, m - 1000)."""
    import synthetic

    for i in (0, 1):
        mx = synthetic.scaling_blobs(i, seed=2)
        m = 3 ** (i + 7)
        assert tuple(mx.X.shape) == (m + 500, 10)
        assert (mx.comp[m:] == -1).all() and (mx.comp[:m] >= 0).all()
        assert float(mx.X[m:].abs().max()) < 50.0
        assert (mx.centres.abs() < 40).all()
    assert synthetic.scaling_sample_size(3 ** 7) == 3 ** 7 - 1000
    assert synthetic.scaling_sample_size(3 ** 15) == 5000
