"""Pins for the oracle's final assignment and objective (Eq. (1); Section 3,
final assignment of the whole data set)."""
import numpy as np


def test_assign_matches_distance_matrix(orc):
    rng = np.random.default_rng(0)
    X = rng.normal(size=(2000, 7)).astype(np.float32)
    Cm = rng.normal(size=(9, 7))
    out = orc.assign_sse(X, Cm)
    Xd = X.astype(np.float64)
    D = ((Xd[:, None, :] - Cm[None]) ** 2).sum(axis=2)
    lab = D.argmin(axis=1)
    assert np.array_equal(out["labels"], lab)
    assert np.array_equal(out["counts"], np.bincount(lab, minlength=9))
    ref = D.min(axis=1)
    assert abs(out["sse"] - ref.sum()) <= 1e-12 * ref.sum()
    assert out["diag"]["n_dist"] == 2000 * 9


def test_degenerate_rows_skipped(orc):
    rng = np.random.default_rng(1)
    X = rng.normal(size=(500, 3)).astype(np.float32)
    Cm = rng.normal(size=(4, 3))
    Cn = Cm.copy()
    Cn[1] = np.nan
    a = orc.assign_sse(X, Cn)
    assert (a["labels"] != 1).all() and a["counts"][1] == 0
    keep = [0, 2, 3]
    b = orc.assign_sse(X, Cm[keep])
    assert np.array_equal(np.array(keep)[b["labels"]], a["labels"])
    assert a["sse"] == b["sse"]
    assert a["diag"]["n_dist"] == 500 * 3


def test_exact_ties_go_to_lowest_index(orc):
    X = np.array([[0.0, 0.0], [1.0, 1.0], [2.0, 0.0]], dtype=np.float32)
    Cm = np.array([[1.0, 0.0], [-1.0, 0.0], [1.0, 0.0]])  # rows 0 and 2 identical
    out = orc.assign_sse(X, Cm, want_margins=True)
    assert out["labels"].tolist() == [0, 0, 0]
    assert out["margins"][0] == 0.0  # exact tie with row 2
    X2 = np.array([[0.0, 0.0]], dtype=np.float32)
    C2 = np.array([[1.0, 0.0], [-1.0, 0.0]])
    assert orc.assign_sse(X2, C2)["labels"].tolist() == [0]


def test_compensated_sum_accuracy(orc):
    """A sum of many terms of very different size: the oracle's compensated
    sum agrees with exact rational arithmetic to ~1 ulp."""
    from fractions import Fraction

    rng = np.random.default_rng(2)
    X = np.concatenate([rng.normal(size=(20000, 1)) * 1e-3, rng.normal(size=(5, 1)) * 1e4])
    X = X.astype(np.float32)
    Cm = np.zeros((1, 1))
    out = orc.assign_sse(X, Cm, want_labels=False)
    exact = sum(Fraction(float(v)) ** 2 for v in X[:, 0].astype(np.float64))
    assert abs(out["sse"] - float(exact)) <= 2e-16 * float(exact)
