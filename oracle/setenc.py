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
sample (K-means++ then Lloyd), compared in normalised coordinates with the
symmetric nearest-neighbour (Chamfer) loss, which does not depend on the
order of the rows:

    L(O, T~) = (1/k) sum_j min_l |O_j - T~_l|^2 + (1/k) sum_l min_j |O_j - T~_l|^2

(argmin ties: lowest index), averaged over the samples of a batch.

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


def chamfer(O, Tn):
    """Symmetric nearest-neighbour loss between O (k x d) and Tn (k' x d),
    and its gradient with respect to O."""
    O = np.asarray(O, dtype=np.float64)
    Tn = np.asarray(Tn, dtype=np.float64)
    k, kt = O.shape[0], Tn.shape[0]
    D = ((O[:, None, :] - Tn[None, :, :]) ** 2).sum(axis=2)  # k x k'
    jl = D.argmin(axis=1)  # nearest target of each proposal
    lj = D.argmin(axis=0)  # nearest proposal of each target
    loss = D[np.arange(k), jl].sum() / k + D[lj, np.arange(kt)].sum() / kt
    g = np.zeros_like(O)
    g += 2.0 / k * (O - Tn[jl])
    np.add.at(g, lj, 2.0 / kt * (O[lj] - Tn))
    return loss, g


def loss_and_grads(params, sets, targets, k: int):
    """Mean Chamfer loss over a batch of (point set, target centroids)
    pairs and the gradient of every parameter."""
    B = len(sets)
    grads = {n: np.zeros_like(params[n]) for n in PARAM_NAMES}
    total = 0.0
    for S, T in zip(sets, targets):
        mu, sigma, St = normalise(S)
        c = encode(params, St)
        Tn = (np.asarray(T, dtype=np.float64) - mu) / sigma
        loss, gO = chamfer(c["o"].reshape(k, -1), Tn)
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
    Chamfer argmin from a tie over the batch: where both are large, the
    loss is smooth around params and central differences are meaningful."""
    m = np.inf
    for S, T in zip(sets, targets):
        mu, sigma, St = normalise(S)
        c = encode(params, St)
        m = min(m, np.abs(c["z1"]).min(), np.abs(c["z2"]).min())
        Tn = (np.asarray(T, dtype=np.float64) - mu) / sigma
        D = ((c["o"].reshape(k, -1)[:, None, :] - Tn[None]) ** 2).sum(axis=2)
        for A in (D, D.T):
            s = np.sort(A, axis=1)
            if s.shape[1] > 1:
                m = min(m, (s[:, 1] - s[:, 0]).min())
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
