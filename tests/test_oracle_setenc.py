"""Pins of the FP64 set-encoder oracle (learned initializer): a forward pass
worked by hand, the linear regime's closed form, the matching
loss's defining properties, and every gradient
entry against central finite differences of the oracle's own loss."""
import numpy as np
import pytest

from oracle import setenc


def _params(d, H, k, rng, scale=1.0):
    shp = setenc.param_shapes(d, k, H)
    return {n: rng.normal(size=shp[n]) * scale / np.sqrt(shp[n][0] if len(shp[n]) == 2 else 4)
            for n in setenc.PARAM_NAMES}


def test_forward_worked_by_hand():
    # S = {0, 2}: mu = 1, sigma = 1, x~ = (-1, 1); z1 = x~ -> h1 = (0, 1);
    # z2 = 2 h1 - 1 = (-1, 1) -> h2 = (0, 1); p = 0.5; o = 4 p + 1 = 3;
    # P = mu + sigma * o = 4
    p = {"W1": np.array([[1.0]]), "b1": np.array([0.0]), "W2": np.array([[2.0]]),
         "b2": np.array([-1.0]), "Wh": np.array([[4.0]]), "bh": np.array([1.0])}
    P = setenc.propose(p, np.array([[0.0], [2.0]]), k=1)
    assert P.shape == (1, 1) and P[0, 0] == 4.0


def test_linear_regime_closed_form():
    """With every pre-activation positive the encoder is affine, and since
    the normalised points have mean zero, the output is ((b1 W2 + b2) Wh +
    bh) whatever the data."""
    rng = np.random.default_rng(0)
    d, H, k = 3, 5, 2
    p = _params(d, H, k, rng)
    p["b1"] = np.full(H, 50.0)
    p["b2"] = np.full(H, 50.0) + np.abs(p["W2"]).sum(0) * 60.0
    S = rng.normal(size=(40, d))
    c = setenc.encode(p, setenc.normalise(S)[2])
    assert (c["z1"] > 0).all() and (c["z2"] > 0).all()
    expect = (p["b1"] @ p["W2"] + p["b2"]) @ p["Wh"] + p["bh"]
    assert np.allclose(c["o"], expect, rtol=1e-12, atol=1e-12)
    mu, sigma, St = setenc.normalise(S)
    assert np.allclose(St.mean(0), 0, atol=1e-14) and np.isclose((St ** 2).sum(1).mean(), 1.0)


def test_greedy_matching_properties():
    rng = np.random.default_rng(1)
    k, d = 6, 3
    T = rng.normal(size=(k, d))
    loss, g = setenc.match_loss(T, T)
    assert loss == 0.0 and not g.any()
    # a shuffled, slightly perturbed copy is matched back to its origin
    perm = rng.permutation(k)
    O = T[perm] + rng.normal(size=(k, d)) * 1e-3
    assert np.array_equal(T[setenc.greedy_match(O, T)], T[perm])
    # on random rows: a permutation, each pair the closest among the rows
    # still free when it was taken (pairs taken in increasing distance)
    O = rng.normal(size=(k, d))
    pi = setenc.greedy_match(O, T)
    assert sorted(pi) == list(range(k))
    D = ((O[:, None, :] - T[None]) ** 2).sum(axis=2)
    used_j, used_l = set(), set()
    for j in np.argsort(D[np.arange(k), pi], kind="stable"):
        for jj in range(k):
            for ll in range(k):
                if jj not in used_j and ll not in used_l:
                    assert D[j, pi[j]] <= D[jj, ll]
        used_j.add(j)
        used_l.add(pi[j])
    loss, g = setenc.match_loss(O, T)
    assert np.isclose(loss, sum(((O[j] - T[pi[j]]) ** 2).sum() for j in range(k)) / k)
    # relabelling proposals or targets relabels the pairing, not the loss
    q = rng.permutation(k)
    assert np.isclose(setenc.match_loss(O[q], T)[0], loss, rtol=1e-14)
    assert np.isclose(setenc.match_loss(O, T[q])[0], loss, rtol=1e-14)
    # one centre: the squared distance
    l1, g1 = setenc.match_loss(O[:1], T[:1])
    assert np.isclose(l1, ((O[0] - T[0]) ** 2).sum()) and np.allclose(g1, 2 * (O[:1] - T[:1]))


def _batch(rng, d, k, B=2, n=7):
    sets = [rng.normal(size=(n, d)) * 2 + rng.normal(size=d) for _ in range(B)]
    targets = [S[rng.choice(n, k, replace=False)] + rng.normal(size=(k, d)) * 0.1 for S in sets]
    return sets, targets


def test_gradients_match_central_differences():
    d, H, k = 3, 8, 2
    for seed in range(50):  # first batch whose loss is smooth around the parameters
        rng = np.random.default_rng(seed)
        p = _params(d, H, k, rng)
        sets, targets = _batch(rng, d, k)
        if setenc.min_kink_margin(p, sets, targets, k) > 1e-3:
            break
    else:
        pytest.fail("no smooth batch found")
    loss, g = setenc.loss_and_grads(p, sets, targets, k)
    h = 1e-6
    gmax = max(np.abs(g[n]).max() for n in setenc.PARAM_NAMES)
    for n in setenc.PARAM_NAMES:
        fd = np.zeros_like(p[n])
        for ix in np.ndindex(p[n].shape):
            old = p[n][ix]
            p[n][ix] = old + h
            lp = setenc.loss_and_grads(p, sets, targets, k)[0]
            p[n][ix] = old - h
            lm = setenc.loss_and_grads(p, sets, targets, k)[0]
            p[n][ix] = old
            fd[ix] = (lp - lm) / (2 * h)
        err = np.abs(fd - g[n])
        assert (err <= 1e-6 * (np.abs(g[n]) + 1e-3 * gmax)).all(), (n, err.max())
        assert np.abs(g[n]).max() > 0 or n == "b1"


def test_acceptance_rule_and_objective():
    rng = np.random.default_rng(2)
    S = rng.normal(size=(30, 2))
    C = S[:3]
    f = setenc.sample_objective(S, C)
    brute = sum(min(((x - c) ** 2).sum() for c in C) for x in S)
    assert np.isclose(f, brute, rtol=1e-14)
    assert setenc.accept(f, f) and setenc.accept(f, f * 2) and not setenc.accept(f * 2, f)
