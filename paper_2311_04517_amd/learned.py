"""Training and use of the learned initializer (set encoder).

Training pairs are made by the method itself: each training sample is
clustered from a cold start (K-means++ seeding, then Lloyd to the stop
rule, Section 3 and Section 6.5) and the converged centroids are the
target of the encoder's proposal for that sample.  Every numeric step runs
in the library's kernels (``hpc_setenc_grad`` / ``hpc_setenc_adam`` /
``hpc_lloyd_batch``); this module only schedules them.
"""
from __future__ import annotations

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
