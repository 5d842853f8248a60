"""Training and use of the learned initializer (set encoder).

Training pairs are made by the method itself: each training sample is
clustered from a cold start (K-means++ seeding, then Lloyd to the stop
rule, Section 3 and Section 6.5) and the converged centroids are the
target of the encoder's proposal for that sample.  Every numeric step runs
in the library's kernels (``hpc_setenc_grad`` / ``hpc_setenc_adam`` /
``hpc_lloyd_batch``); this module only schedules them.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import api


def sub_desc(desc, rows):
    """Descriptor array of the samples ``rows`` of ``desc`` (offsets kept,
    so they still index the full idx / target arrays)."""
    out = (api.SampleDesc * len(rows))()
    for i, b in enumerate(rows):
        out[i] = desc[int(b)]
    return out


def method_targets(X, idx, desc, c_len, *, precision=api.PREC_FP32, max_iter=300, rel_tol=1e-4):
    """Converged centroids of a cold start on every sample (the targets)."""
    T = torch.full((c_len,), float("nan"), dtype=torch.float32, device=X.device)
    f, it, _ = api.lloyd_batch(X, idx, desc, T, max_iter=max_iter, rel_tol=rel_tol,
                               precision=precision)
    return T, f, it


def train(model: api.SetEncoder, X, idx, desc, T, *, steps: int, batch: int, lr: float = 1e-3,
          seed: int = 0, lr_final: float | None = None):
    """Adam on random batches of the training samples.  Returns the loss of
    every step (read back once at the end)."""
    rng = np.random.default_rng(seed)
    n = len(desc)
    losses = torch.empty(steps, dtype=torch.float64, device=X.device)
    for t in range(steps):
        rows = rng.choice(n, size=min(batch, n), replace=False)
        model.grad(X, idx, sub_desc(desc, rows), T, loss=losses[t:t + 1])
        a = lr if lr_final is None else lr * (lr_final / lr) ** (t / max(1, steps - 1))
        model.adam(a)
    return losses.cpu().numpy()


def heldout_loss(model: api.SetEncoder, X, idx, desc, T, batch: int):
    """Mean matching loss over held-out samples (no parameter update)."""
    tot, n = 0.0, len(desc)
    for a in range(0, n, batch):
        rows = np.arange(a, min(n, a + batch))
        loss = model.grad(X, idx, sub_desc(desc, rows), T)
        tot += loss.item() * len(rows)
    return tot / n


class Pairs:
    """Training (or held-out) pairs in device memory: for every sample, the
    points the encoder reads (the first n_enc of its rows, as the kernels
    take them) and the centroids the method converged to on the whole
    sample.  Sample b occupies rows [b n_enc, (b + 1) n_enc) of ``X`` and
    the k x d block at b k d of ``T``."""

    def __init__(self, d: int, k: int, n_enc: int):
        self.d, self.k, self.n_enc = d, k, n_enc
        self._x, self._t = [], []
        self.X = self.T = self.idx = self.desc = None
        self.n = 0

    def add(self, X, idx, desc, T):
        """Append the samples of ``desc`` (their rows through ``idx``, their
        targets in ``T`` at each c_offset); every s >= n_enc."""
        n, e, k, d = len(desc), self.n_enc, self.k, self.d
        io = torch.tensor([desc[b].idx_offset for b in range(n)], dtype=torch.int64,
                          device=X.device)
        co = torch.tensor([desc[b].c_offset for b in range(n)], dtype=torch.int64,
                          device=X.device)
        if min(desc[b].s for b in range(n)) < e:
            raise ValueError("every sample needs at least n_enc points")
        rows = idx[io[:, None] + torch.arange(e, device=X.device)]
        self._x.append(X[rows.reshape(-1)].reshape(n * e, d))
        self._t.append(T[co[:, None] + torch.arange(k * d, device=X.device)].reshape(-1))

    def finish(self):
        self.X = torch.cat(self._x)
        self.T = torch.cat(self._t)
        self._x, self._t = [], []
        self.n = self.X.shape[0] // self.n_enc
        self.idx = torch.arange(self.X.shape[0], dtype=torch.int64, device=self.X.device)
        self.desc, _, _ = api.make_desc([self.n_enc] * self.n, [self.k] * self.n, seed=0,
                                        sample_id=range(self.n), d=self.d)
        return self


def lr_at(step: int, total: int, lr: float, lr_min: float, warmup: int) -> float:
    """Learning rate of step ``step`` of ``total``: linear warm-up over
    ``warmup`` steps to ``lr``, then a cosine decay to ``lr_min``."""
    if step < warmup:
        return lr * (step + 1) / warmup
    t = (step - warmup) / max(1, total - warmup - 1)
    return lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * min(1.0, t)))


def fit(model: api.SetEncoder, train: Pairs, held: Pairs | None, *, epochs: int, batch: int,
        lr: float = 2e-3, lr_min: float = 2e-5, warmup: int = 200, seed: int = 0,
        on_epoch=None):
    """Adam over ``epochs`` shuffled passes of the training pairs with the
    schedule of ``lr_at``.  Returns the curve: per epoch (0 = before
    training) the mean training loss of its steps and the held-out loss;
    ``on_epoch`` (nullable) is called with each entry as it is made."""
    rng = np.random.default_rng(seed)
    per = max(1, train.n // batch)
    total = epochs * per
    curve = [{"epoch": 0, "step": 0, "train": None,
              "heldout": heldout_loss(model, held.X, held.idx, held.desc, held.T, batch)
              if held is not None else None}]
    step = 0
    for ep in range(epochs):
        perm = rng.permutation(train.n)
        losses = torch.empty(per, dtype=torch.float64, device=train.X.device)
        for i in range(per):
            rows = perm[i * batch:(i + 1) * batch]
            model.grad(train.X, train.idx, sub_desc(train.desc, rows), train.T,
                       loss=losses[i:i + 1])
            model.adam(lr_at(step, total, lr, lr_min, warmup))
            step += 1
        curve.append({"epoch": ep + 1, "step": step, "train": losses.mean().item(),
                      "heldout": heldout_loss(model, held.X, held.idx, held.desc, held.T, batch)
                      if held is not None else None})
        if on_epoch is not None:
            on_epoch(curve[-1])
    return curve


def evaluate(model: api.SetEncoder, X, idx, desc, c_len, *, precision=api.PREC_FP32,
             max_iter: int = 300, rel_tol: float = 1e-4):
    """The learned initializer against K-means++ on cold samples: the
    seeding choice (proposal where its sample objective is no larger than
    the K-means++ seeding's), then Lloyd to the stop rule from the chosen
    seeds, from the K-means++ seeds alone, and from the raw proposals.
    Returns per-sample arrays (host numpy): accepted, f_prop, f_kpp, and
    for each start its passes and final objective."""
    dev = X.device
    C = torch.empty(c_len, dtype=torch.float32, device=dev)
    C_kpp = torch.empty_like(C)
    C, C_kpp, f_prop, f_kpp, acc = model.learned_seed(X, idx, desc, C, precision=precision,
                                                      C_kpp=C_kpp)
    P = model.propose(X, idx, desc, torch.empty_like(C))
    out = {"accepted": acc.cpu().numpy(), "f_prop": f_prop.cpu().numpy(),
           "f_kpp": f_kpp.cpu().numpy()}
    for name, C0 in (("learned", C), ("kmeanspp", C_kpp), ("proposal", P)):
        Cw = C0.clone()
        f, it, _ = api.lloyd_batch(X, idx, desc, Cw, max_iter=max_iter, rel_tol=rel_tol,
                                   precision=precision)
        out[name] = {"passes": it.cpu().numpy(), "f": f.cpu().numpy()}
    return out


def summarize(ev: dict) -> dict:
    """Means and ratios of ``evaluate``'s per-sample results."""
    kp = ev["kmeanspp"]
    res = {"samples": int(len(ev["accepted"])),
           "accepted_frac": float(np.mean(ev["accepted"])),
           "seed_objective_ratio_median": float(np.median(ev["f_prop"] / ev["f_kpp"])),
           "seed_objective_ratio_min": float(np.min(ev["f_prop"] / ev["f_kpp"]))}
    for name in ("learned", "kmeanspp", "proposal"):
        r = ev[name]
        ratio = r["f"] / kp["f"]
        res[name] = {"passes_mean": float(np.mean(r["passes"])),
                     "passes_max": int(np.max(r["passes"])),
                     "final_f_over_kmeanspp_mean": float(np.mean(ratio)),
                     "better_frac": float(np.mean(ratio < 1 - 1e-12)),
                     "worse_frac": float(np.mean(ratio > 1 + 1e-12))}
    return res
