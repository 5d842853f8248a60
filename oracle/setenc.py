"""FP64 reference of the learned initializer (set encoder) -- TEST
INFRASTRUCTURE ONLY.

Not part of the product path: only tests/, ``__graft_entry__.smoke()`` and
the benchmark's CPU baseline may import this module.

The paper seeds every cold sample with K-means++ (Section 3; three
candidates per new centre, Section 6.5).  The learned initializer proposes
the k starting centroids of a sample from the sample itself with a set
encoder, and the proposal replaces the K-means++ seeding only when its
sample objective (Eq. (1) restricted to the sample) is no larger than that
of the K-means++ seeding on the same sample.  The model:

    normalisation  mu = mean of the points, sigma = sqrt(mean |x - mu|^2),
                   x~ = (x - mu) / sigma
    per point      z1 = x~ W1 + b1,  h1 = relu(z1)       (d -> H)
                   z2 = h1 W2 + b2,  h2 = relu(z2)       (H -> H)
    pooling        p = mean over the points of h2        (H)
    head           o = p Wh + bh                          (H -> k*d)
    proposal       P = mu + sigma * reshape(o, k, d)

Training target: the centroids T the method converges to on the same
sample (K-means++ then Lloyd), compared in normalised coordinates after a
one-to-one greedy matching, which does not depend on the order of the rows:
repeatedly pair the closest proposal row O_j and target row T~_l among the
rows not yet paired (ties: lowest j, then lowest l), giving a permutation pi;

    L(O, T~) = (1/k) sum_j |O_j - T~_pi(j)|^2,

averaged over the samples of a batch (pi is held fixed when
differentiating).

Every function is plain numpy in float64; the encoder's gradient is the
chain rule written out layer by layer.
"""
from __future__ import annotations

import numpy as np

PARAM_NAMES = ("W1", "b1", "W2", "b2", "Wh", "bh")


def param_shapes(d: int, k: int, H: int = 256) -> dict:
    return {"W1": (d, H), "b1": (H,), "W2": (H, H), "b2": (H,), "Wh": (H, k * d),
            "bh": (k * d,)}


def normalise(S):
    """(mu, sigma, S~) of one point set."""
    S = np.asarray(S, dtype=np.float64)
    mu = S.mean(axis=0)
    sigma = np.sqrt(((S - mu) ** 2).sum(axis=1).mean())
    if not sigma > 0:
        sigma = 1.0
    return mu, sigma, (S - mu) / sigma


def encode(params, St):
    """Forward pass on one normalised set St (n x d): returns the cache of
    every intermediate (z1, h1, z2, h2, p, o)."""
    z1 = St @ params["W1"] + params["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ params["W2"] + params["b2"]
    h2 = np.maximum(z2, 0.0)
    p = h2.mean(axis=0)
    o = p @ params["Wh"] + params["bh"]
    return dict(St=St, z1=z1, h1=h1, z2=z2, h2=h2, p=p, o=o)


def propose(params, S, k: int):
    """Proposal P (k x d) for the point set S."""
    mu, sigma, St = normalise(S)
    o = encode(params, St)["o"]
    return mu + sigma * o.reshape(k, -1)


def greedy_match(O, Tn):
    """The greedy one-to-one pairing pi (pi[j] = target of proposal j) of
    two k x d row sets by squared distance."""
    O = np.asarray(O, dtype=np.float64)
    Tn = np.asarray(Tn, dtype=np.float64)
    k = O.shape[0]
    D = ((O[:, None, :] - Tn[None, :, :]) ** 2).sum(axis=2)
    pi = np.full(k, -1)
    free_j = np.ones(k, dtype=bool)
    free_l = np.ones(k, dtype=bool)
    for _ in range(k):
        M = np.where(free_j[:, None] & free_l[None, :], D, np.inf)
        j, l = np.unravel_index(np.argmin(M), M.shape)  # first minimum in row-major order
        pi[j] = l
        free_j[j] = False
        free_l[l] = False
    return pi


def match_loss(O, Tn):
    """Matching loss of one sample and its gradient with respect to O."""
    O = np.asarray(O, dtype=np.float64)
    Tn = np.asarray(Tn, dtype=np.float64)
    k = O.shape[0]
    pi = greedy_match(O, Tn)
    E = O - Tn[pi]
    return (E ** 2).sum() / k, 2.0 / k * E


def loss_and_grads(params, sets, targets, k: int):
    """Mean matching loss over a batch of (point set, target centroids)
    pairs and the gradient of every parameter."""
    B = len(sets)
    grads = {n: np.zeros_like(params[n]) for n in PARAM_NAMES}
    total = 0.0
    for S, T in zip(sets, targets):
        mu, sigma, St = normalise(S)
        c = encode(params, St)
        Tn = (np.asarray(T, dtype=np.float64) - mu) / sigma
        loss, gO = match_loss(c["o"].reshape(k, -1), Tn)
        total += loss / B
        do = gO.ravel() / B
        grads["Wh"] += np.outer(c["p"], do)
        grads["bh"] += do
        dp = params["Wh"] @ do
        n = St.shape[0]
        dz2 = (c["z2"] > 0) * (dp / n)[None, :]
        grads["W2"] += c["h1"].T @ dz2
        grads["b2"] += dz2.sum(axis=0)
        dh1 = dz2 @ params["W2"].T
        dz1 = (c["z1"] > 0) * dh1
        grads["W1"] += St.T @ dz1
        grads["b1"] += dz1.sum(axis=0)
    return total, grads


def min_kink_margin(params, sets, targets, k: int) -> float:
    """Smallest distance of any ReLU pre-activation from 0 and of any
    greedy-matching choice from a tie over the batch: where both are large,
    the loss is smooth around params and central differences are
    meaningful."""
    m = np.inf
    for S, T in zip(sets, targets):
        mu, sigma, St = normalise(S)
        c = encode(params, St)
        m = min(m, np.abs(c["z1"]).min(), np.abs(c["z2"]).min())
        Tn = (np.asarray(T, dtype=np.float64) - mu) / sigma
        O = c["o"].reshape(k, -1)
        D = ((O[:, None, :] - Tn[None]) ** 2).sum(axis=2)
        pi = greedy_match(O, Tn)
        free_j = np.ones(k, dtype=bool)
        free_l = np.ones(k, dtype=bool)
        for j in np.argsort(D[np.arange(k), pi], kind="stable"):
            M = np.where(free_j[:, None] & free_l[None, :], D, np.inf)
            M[j, pi[j]] = np.inf
            m = min(m, M.min() - D[j, pi[j]])
            free_j[j] = False
            free_l[pi[j]] = False
    return float(m)


def sample_objective(S, C):
    """f(C, S) = sum_i min_j |x_i - c_j|^2 (Eq. (1) on the sample)."""
    S = np.asarray(S, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    D = ((S[:, None, :] - C[None, :, :]) ** 2).sum(axis=2)
    return float(D.min(axis=1).sum())


def accept(f_prop: float, f_kpp: float) -> bool:
    """The proposal replaces the K-means++ seeding iff it is at least as
    good on the sample."""
    return f_prop <= f_kpp
