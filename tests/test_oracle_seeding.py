"""Pins for the oracle's K-means++ seeding (Section 3: K-means++ initialises
the first sample and re-initialises degenerate centroids; Section 6.5: three
candidate points per new centroid, the one of least potential is kept)."""
import itertools

import numpy as np
import pytest
from scipy import stats

from tests.test_oracle_rng import _numpy_block

TAG_SEED = 1


def _pot(P, D2, j):
    dj = ((P - P[j]) ** 2).sum(axis=1)
    return np.minimum(D2, dj).sum()


def _greedy_choice_probs(P, D2, n_cand):
    """Exact probability of each point being chosen by one greedy D^2 step:
    sum over all ordered candidate tuples of the product of D^2/W, with the
    winner the least potential (ties to the earlier draw)."""
    W = D2.sum()
    p = D2 / W
    pots = np.array([_pot(P, D2, j) for j in range(len(P))])
    probs = np.zeros(len(P))
    for tup in itertools.product(range(len(P)), repeat=n_cand):
        w = np.prod([p[j] for j in tup])
        if w == 0:
            continue
        best = tup[0]
        for j in tup[1:]:
            if pots[j] < pots[best]:
                best = j
        probs[best] += w
    return probs


@pytest.mark.parametrize("n_cand", [1, 3])
def test_d2_step_distribution(orc, n_cand):
    """One D^2 step after one valid centre: observed choice frequencies over
    many independent streams match the exact law (chi-square)."""
    P = np.array([[0.0, 0.0], [1.0, 0.0], [3.0, 1.0], [0.5, 2.5], [4.0, 4.0]], dtype=np.float32)
    valid = np.array([[0.2, 0.1]])
    Cin = np.vstack([valid, np.full((1, 2), np.nan)])
    D2 = ((P.astype(np.float64) - valid) ** 2).sum(axis=1)
    probs = _greedy_choice_probs(P.astype(np.float64), D2, n_cand)
    idx = np.arange(5, dtype=np.int64)
    n = 40_000
    counts = np.zeros(5)
    for call in range(n):
        C, chosen, _ = orc.kmeanspp(P, idx, 2, seed=17, sample_id=3, call_id=call, n_cand=n_cand,
                                    C=Cin)
        assert chosen[0] == -1
        counts[chosen[1]] += 1
        assert np.array_equal(C[1], P[chosen[1]].astype(np.float64))
        assert np.array_equal(C[0], valid[0])
    exp = probs * n
    mask = exp > 0
    assert counts[~mask].sum() == 0
    chi2 = ((counts[mask] - exp[mask]) ** 2 / exp[mask]).sum()
    assert stats.chi2.sf(chi2, mask.sum() - 1) > 1e-6, (counts, exp)


def test_first_centre_uniform_and_stream_layout(orc):
    """With no valid row the first centre is sample point floor(r*s/2^64),
    r = word 0 of block 0 of stream (seed, SEED) / (0, sample, call, 0)."""
    rng = np.random.default_rng(0)
    s = 7
    P = rng.normal(size=(s, 3)).astype(np.float32)
    idx = np.arange(s, dtype=np.int64)
    counts = np.zeros(s)
    for call in range(3000):
        _, chosen, _ = orc.kmeanspp(P, idx, 1, seed=5, sample_id=2, call_id=call)
        r = int(_numpy_block([0, 2, call, 0], [5, TAG_SEED])[0])
        assert chosen[0] == (r * s) >> 64
        counts[chosen[0]] += 1
    chi2 = ((counts - 3000 / s) ** 2 / (3000 / s)).sum()
    assert stats.chi2.sf(chi2, s - 1) > 1e-6


def test_zero_weight_points_never_chosen(orc):
    """Points that coincide with an existing centre have D^2 = 0 and are
    never drawn."""
    P = np.array([[0, 0]] * 6 + [[5, 5], [6, 5]], dtype=np.float32)
    idx = np.arange(len(P), dtype=np.int64)
    Cin = np.array([[0.0, 0.0], [np.nan, np.nan]])
    for call in range(500):
        _, chosen, g = orc.kmeanspp(P, idx, 2, seed=1, call_id=call, C=Cin)
        assert chosen[1] in (6, 7)
        assert g["n_zero_weight"] == 0


def test_zero_total_weight_falls_back_to_uniform(orc):
    """Every point coincides with a valid centre (W = 0): the row takes the
    point floor(r*s/2^64), r = word 0 of block 1."""
    P = np.zeros((9, 2), dtype=np.float32)
    idx = np.arange(9, dtype=np.int64)
    Cin = np.array([[0.0, 0.0], [np.nan, np.nan]])
    for call in range(50):
        _, chosen, g = orc.kmeanspp(P, idx, 2, seed=8, sample_id=1, call_id=call, C=Cin)
        r = int(_numpy_block([1, 1, call, 0], [8, TAG_SEED])[0])
        assert chosen[1] == (r * 9) >> 64
        assert g["n_zero_weight"] == 1


def test_seeding_k_equals_s_is_a_permutation(orc):
    """With k = s distinct points every point becomes a centre exactly once
    (a chosen point has D^2 = 0 afterwards)."""
    rng = np.random.default_rng(3)
    P = rng.normal(size=(12, 4)).astype(np.float32)
    idx = np.arange(12, dtype=np.int64)
    for call in range(20):
        C, chosen, _ = orc.kmeanspp(P, idx, 12, seed=3, call_id=call)
        assert sorted(chosen.tolist()) == list(range(12))
        assert np.array_equal(C, P[chosen].astype(np.float64))


def test_valid_rows_kept_and_distance_count(orc):
    """Valid rows are untouched; cost is s per valid row for the initial D^2
    and n_cand * s per seeded row; a cold start costs s*(1 + n_cand*(k-1))."""
    rng = np.random.default_rng(4)
    s, d, k = 300, 5, 6
    P = rng.normal(size=(s, d)).astype(np.float32)
    idx = np.arange(s, dtype=np.int64)
    _, _, g = orc.kmeanspp(P, idx, k, seed=2)
    assert g["n_dist"] == s * (1 + 3 * (k - 1))
    Cin = np.full((k, d), np.nan)
    Cin[1] = 1.0
    Cin[4] = -1.0
    C, chosen, g = orc.kmeanspp(P, idx, k, seed=2, C=Cin)
    assert np.array_equal(C[1], Cin[1]) and np.array_equal(C[4], Cin[4])
    assert chosen[1] == -1 and chosen[4] == -1
    assert all(chosen[j] >= 0 for j in (0, 2, 3, 5))
    assert g["n_dist"] == s * 2 + 3 * s * 4
    assert not np.isnan(C).any()


def test_seeded_centres_are_distinct_sample_points(orc):
    rng = np.random.default_rng(5)
    P = rng.normal(size=(500, 8)).astype(np.float32)
    idx = rng.integers(0, 500, size=200).astype(np.int64)
    C, chosen, _ = orc.kmeanspp(P, idx, 10, seed=11, sample_id=4)
    assert len(set(idx[chosen].tolist())) == 10
    assert np.array_equal(C, P[idx[chosen]].astype(np.float64))
