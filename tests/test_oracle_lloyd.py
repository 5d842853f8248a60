"""Pins for the oracle's K-means local search and worker loop
(Eq. (1); Algorithm 1 assign/update; Section 3 and Algorithm 3 for the
degenerate re-initialisation and keep-the-best; Section 6.5 stop rule)."""
import itertools

import numpy as np
import pytest


def _sse_of_labels(P, lab, k):
    tot = 0.0
    for j in range(k):
        Q = P[lab == j]
        if len(Q):
            tot += ((Q - Q.mean(axis=0)) ** 2).sum()
    return tot


def _brute_force_opt(P, k):
    """Exact MSSC optimum by enumerating all k^m labelings."""
    m = len(P)
    best = np.inf
    for lab in itertools.product(range(k), repeat=m):
        if lab[0] != 0:  # symmetry: first point in cluster 0
            continue
        best = min(best, _sse_of_labels(P, np.array(lab), k))
    return best


def _dp_1d_opt(x, k):
    """Exact 1-D MSSC optimum: optimal clusters are contiguous in sorted
    order (dynamic programming over prefix sums)."""
    x = np.sort(np.asarray(x, dtype=np.float64))
    m = len(x)
    s1 = np.concatenate([[0.0], np.cumsum(x)])
    s2 = np.concatenate([[0.0], np.cumsum(x * x)])

    def cost(a, b):  # points a..b-1
        n = b - a
        mu = (s1[b] - s1[a]) / n
        return max(0.0, (s2[b] - s2[a]) - n * mu * mu)

    D = np.full((k + 1, m + 1), np.inf)
    D[0, 0] = 0.0
    for c in range(1, k + 1):
        for b in range(1, m + 1):
            D[c, b] = min((D[c - 1, a] + cost(a, b) for a in range(c - 1, b)), default=np.inf)
    return D[k, m]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_lower_bound_and_optimum(orc, seed):
    rng = np.random.default_rng(seed)
    m, k = 10, 3
    P = rng.normal(size=(m, 2)).astype(np.float32)
    fstar = _brute_force_opt(P.astype(np.float64), k)
    idx = np.arange(m, dtype=np.int64)
    for sd in range(5):
        r = orc.lloyd(P, idx, k, seed=sd)
        assert r.f >= fstar - 1e-12
    # well separated: three tight groups far apart -> Lloyd reaches f*
    centres = np.array([[0, 0], [50, 0], [0, 50]], dtype=np.float64)
    Q = (centres[rng.integers(0, 3, size=m)] + 0.3 * rng.normal(size=(m, 2))).astype(np.float32)
    Q[:3] = (centres + 0.3 * rng.normal(size=(3, 2))).astype(np.float32)
    fq = _brute_force_opt(Q.astype(np.float64), k)
    r = orc.lloyd(Q, idx, k, seed=seed, rel_tol=0.0, max_iter=50)
    assert abs(r.f - fq) <= 1e-9 * fq


def test_1d_dynamic_programming_bound(orc):
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.normal(c, 1.0, 40) for c in (0, 30, 60, 90)]).astype(np.float32)
    P = x[:, None]
    idx = np.arange(len(x), dtype=np.int64)
    fstar = _dp_1d_opt(x, 4)
    r = orc.lloyd(P, idx, 4, seed=1, rel_tol=0.0, max_iter=100)
    assert abs(r.f - fstar) <= 1e-9 * fstar
    # overlapping data: Lloyd never beats the optimum
    y = rng.normal(size=150).astype(np.float32)
    fy = _dp_1d_opt(y, 3)
    for sd in range(4):
        ry = orc.lloyd(y[:, None], np.arange(150, dtype=np.int64), 3, seed=sd)
        assert ry.f >= fy - 1e-12


def test_k1_closed_form(orc):
    """k = 1: pass 1 uses the seeded point, the update gives the mean, pass 2
    gives the total scatter, pass 3 changes nothing -> stop after 3 passes."""
    rng = np.random.default_rng(9)
    P = rng.normal(3.0, 2.0, size=(400, 6)).astype(np.float32)
    idx = rng.integers(0, 400, size=250).astype(np.int64)
    r = orc.lloyd(P, idx, 1, seed=4)
    S = P[idx].astype(np.float64)
    mu = S.mean(axis=0)
    scatter = ((S - mu) ** 2).sum()
    assert r.iters == 3
    assert np.allclose(r.C[0], mu, rtol=0, atol=1e-12)
    assert abs(r.f - scatter) <= 1e-12 * scatter


def _f_sequence(orc, P, idx, k, C0, seed, T):
    """f after t passes, t = 1..T (the run is deterministic, so truncating
    max_iter reveals the trajectory)."""
    return [orc.lloyd(P, idx, k, C0, seed=seed, max_iter=t, rel_tol=0.0).f for t in range(1, T + 1)]


def test_monotone_objective_including_reseed(orc):
    rng = np.random.default_rng(11)
    P = np.concatenate([rng.normal(c, 1.0, size=(100, 3)) for c in (0.0, 8.0, 16.0)]).astype(
        np.float32)
    idx = np.arange(300, dtype=np.int64)
    # row 2 is far from every point: it receives no point in pass 1, becomes
    # degenerate and is re-seeded at the top of pass 2
    C0 = np.array([[0.0, 0, 0], [1.0, 1, 1], [1e3, 1e3, 1e3]])
    fs = _f_sequence(orc, P, idx, 3, C0, 5, 12)
    for a, b in zip(fs, fs[1:]):
        assert b <= a * (1 + 1e-12)
    r2 = orc.lloyd(P, idx, 3, C0, seed=5, max_iter=2, rel_tol=0.0)
    assert r2.diag["n_seed_calls"] == 1 and r2.diag["n_seeded_rows"] == 1
    assert not np.isnan(r2.C).any()
    assert fs[1] < 0.8 * fs[0]


def test_fixed_point_and_sse_identity(orc):
    rng = np.random.default_rng(12)
    P = rng.normal(size=(600, 4)).astype(np.float32)
    idx = np.arange(600, dtype=np.int64)
    r = orc.lloyd(P, idx, 5, seed=3, rel_tol=0.0, max_iter=300)
    S = P.astype(np.float64)
    lab = r.labels
    for j in range(5):
        assert np.allclose(r.C[j], S[lab == j].mean(axis=0), rtol=0, atol=1e-12)
    dist = ((S[:, None, :] - r.C[None, :, :]) ** 2).sum(axis=2)
    assert np.array_equal(np.argmin(dist, axis=1), lab)
    # SSE identity at the fixed point: sum|x-c_a|^2 = sum|x|^2 - sum_j n_j |c_j|^2
    out = orc.assign_sse(P, r.C)
    n = np.bincount(lab, minlength=5)
    ident = (S ** 2).sum() - (n * (r.C ** 2).sum(axis=1)).sum()
    assert abs(out["sse"] - ident) <= 1e-10 * out["sse"]
    assert abs(out["sse"] - r.f) <= 1e-12 * r.f


def test_stop_rule(orc):
    """Stops at the first pass t >= 2 whose relative improvement is below
    rel_tol, or at max_iter."""
    rng = np.random.default_rng(13)
    P = rng.normal(size=(500, 3)).astype(np.float32)
    idx = np.arange(500, dtype=np.int64)
    fs = _f_sequence(orc, P, idx, 6, None, 7, 40)
    for tol in (1e-1, 1e-2, 1e-4):
        r = orc.lloyd(P, idx, 6, seed=7, rel_tol=tol)
        expect = next((t for t in range(2, 41) if (fs[t - 2] - fs[t - 1]) < tol * fs[t - 2]), None)
        assert expect is not None and r.iters == expect
        assert r.f == fs[r.iters - 1]
    assert orc.lloyd(P, idx, 6, seed=7, max_iter=4, rel_tol=0.0).iters == 4


def test_zero_objective_stops(orc):
    P = np.repeat(np.array([[1.0, 2.0], [5.0, 5.0]], dtype=np.float32), 10, axis=0)
    r = orc.lloyd(P, np.arange(20, dtype=np.int64), 2, seed=0)
    assert r.f == 0.0 and r.iters == 1


def test_separated_mixture_end_to_end(orc):
    """Components >= 12 sigma apart: the worker loop recovers the component
    partition, and its objective is within a few percent of that partition's
    optimum (about d*sigma^2*m)."""
    rng = np.random.default_rng(14)
    k, d, m, sig = 5, 4, 4000, 1.0
    mu = rng.uniform(-100, 100, size=(k, d))
    while min(np.linalg.norm(mu[a] - mu[b]) for a in range(k) for b in range(a)) < 12 * sig:
        mu = rng.uniform(-100, 100, size=(k, d))
    comp = rng.integers(0, k, size=m)
    X = (mu[comp] + sig * rng.normal(size=(m, d))).astype(np.float32)
    w = orc.worker_loop(X, s=500, k=k, n_samples=6, seed=21)
    # the recovered partition is the component partition (up to relabelling)
    pairs = set(zip(comp.tolist(), w["labels"].tolist()))
    assert len(pairs) == k and len({a for a, _ in pairs}) == k and len({b for _, b in pairs}) == k
    # its optimal objective (means of the components) bounds the run from below
    Xd = X.astype(np.float64)
    opt = sum(((Xd[comp == j] - Xd[comp == j].mean(axis=0)) ** 2).sum() for j in range(k))
    assert opt <= w["sse"] <= opt * 1.05
    assert abs(opt / (d * sig**2 * m) - 1) < 0.1
    assert w["f_hat"] == w["f_samples"].min()


def test_keep_best_composition(orc):
    """The worker loop equals its definition written with the oracle's
    sample draw, Lloyd and strict keep-the-best."""
    rng = np.random.default_rng(15)
    X = rng.normal(size=(3000, 3)).astype(np.float32)
    s, k, n, seed = 200, 7, 6, 33
    w = orc.worker_loop(X, s=s, k=k, n_samples=n, seed=seed)
    Cw, fhat = np.full((k, 3), np.nan), np.inf
    for t in range(n):
        idx = orc.draw_sample(3000, s, seed, t)
        r = orc.lloyd(X, idx, k, Cw, seed=seed, sample_id=t)
        assert r.f == w["f_samples"][t] and r.iters == w["iters"][t]
        if r.f < fhat:
            Cw, fhat = r.C, r.f
    assert np.array_equal(Cw, w["C"]) and fhat == w["f_hat"]
    full = orc.assign_sse(X, Cw)
    assert full["sse"] == w["sse"] and np.array_equal(full["labels"], w["labels"])


def test_batch_matches_single_and_threads(orc):
    rng = np.random.default_rng(16)
    X = rng.normal(size=(5000, 4)).astype(np.float32)
    ss = [100, 250, 60, 400]
    ks = [3, 8, 2, 5]
    io = np.concatenate([[0], np.cumsum(ss)[:-1]])
    co = np.concatenate([[0], np.cumsum([k * 4 for k in ks])[:-1]])
    idx = np.concatenate([orc.draw_sample(5000, s, 9, b) for b, s in enumerate(ss)])
    desc = dict(idx_offset=io, s=ss, k=ks, c_offset=co, seed=[9] * 4, sample_id=[0, 1, 2, 3])
    outs = []
    for nt in (1, 3):
        Cb = np.full(sum(k * 4 for k in ks), np.nan)
        o = orc.lloyd_batch(X, idx, desc, Cb, n_threads=nt, want_labels=True)
        outs.append((Cb, o))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1]["f"], outs[1][1]["f"])
    for b in range(4):
        r = orc.lloyd(X, idx[io[b]:io[b] + ss[b]], ks[b], seed=9, sample_id=b)
        assert r.f == outs[0][1]["f"][b] and r.iters == outs[0][1]["iters"][b]
        assert np.array_equal(r.C.ravel(), outs[0][0][co[b]:co[b] + ks[b] * 4])
