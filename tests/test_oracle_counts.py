"""Distance-evaluation structure (Appendix A prints n_d per run).

The paper's counts decompose exactly as
    n_d = m*k + W*s*(1 + 3*(k-1)) + s*k*P
with P the total number of assignment passes: the final assignment of the
whole data set, one cold K-means++ seeding per worker (one pass to the
first centre, three candidate potentials per further centre), and one
distance per point and centroid per pass.  The pin checks (i) that the
printed numbers give an integer P with three candidates and not with other
candidate counts, and (ii) that the oracle's own counter has exactly this
structure on a run without later re-seeding.
"""
import os

import numpy as np

GOLD = os.path.join(os.path.dirname(__file__), "golden", "appendix_distance_counts.txt")


def _rows():
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        ds, m, s, st, W, k, nd = line.split()
        yield ds, int(m), int(s), st, int(W), int(k), int(nd)


def _passes(m, s, W, k, nd, n_cand, first_pass=1):
    rest = nd - m * k - W * s * (first_pass + n_cand * (k - 1))
    return rest / (s * k)


def test_paper_counts_integral_with_three_candidates():
    rows = list(_rows())
    assert len(rows) == 28
    for ds, m, s, st, W, k, nd in rows:
        P = _passes(m, s, W, k, nd, 3)
        assert P == int(P) and P > 0, (ds, st, k, P)


def test_other_candidate_counts_do_not_fit():
    rows = list(_rows())
    for n_cand in (1, 2, 4, 5):
        assert any(_passes(m, s, W, k, nd, n_cand) % 1 != 0 for _, m, s, _, W, k, nd in rows)
    # without the pass to the first centre the counts do not fit either
    assert any(_passes(m, s, W, k, nd, 3, first_pass=0) % 1 != 0 for _, m, s, _, W, k, nd in rows)


def test_oracle_counter_has_the_same_structure(orc):
    rng = np.random.default_rng(0)
    k, d, m, s = 4, 3, 6000, 400
    mu = np.array([[0, 0, 0], [40, 0, 0], [0, 40, 0], [0, 0, 40]], dtype=np.float64)
    X = (mu[rng.integers(0, k, size=m)] + rng.normal(size=(m, d))).astype(np.float32)
    w = orc.worker_loop(X, s=s, k=k, n_samples=5, seed=1)
    g = w["diag"]
    assert g["n_seed_calls"] == 1  # only the cold start of sample 0
    P = int(w["iters"].sum())
    assert g["n_dist"] == m * k + s * (1 + 3 * (k - 1)) + s * k * P
