"""Worker loops of the method built from the C-ABI calls.

``worker_loop`` is one worker of Algorithm 3 (the sequential form of
Section 3).  ``strategy_rounds`` runs W workers per round as one batched
launch: competitive (Algorithm 3: each worker restarts from its own
incumbent), cooperative (Algorithm 4: every worker restarts from the best
incumbent) and hybrid (Algorithm 5: competitive rounds, then cooperative
rounds).  All arithmetic runs in the library's kernels; torch only holds
memory and copies incumbents between buffers.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import api


@dataclass
class WorkerResult:
    C: torch.Tensor          # k x d incumbent
    f_hat: torch.Tensor      # [1] float64
    f_samples: torch.Tensor  # n_samples float64
    iters: torch.Tensor      # n_samples int32
    labels: torch.Tensor | None
    counts: torch.Tensor | None
    sse: torch.Tensor | None


def worker_loop(X: torch.Tensor, *, s: int, k: int, n_samples: int, seed: int, max_iter=300,
                rel_tol=1e-4, precision=api.PREC_FP32, final_assign=True) -> WorkerResult:
    """C_w <- all degenerate; for t < n_samples: sample t, K-means from C_w
    (degenerate rows re-seeded first), keep the best; then assign X."""
    m, d = X.shape
    dev = X.device
    C_w = torch.full((k, d), float("nan"), dtype=torch.float32, device=dev)
    f_hat = torch.full((1,), float("inf"), dtype=torch.float64, device=dev)
    C = torch.empty((k, d), dtype=torch.float32, device=dev)
    idx = torch.empty(s, dtype=torch.int64, device=dev)
    f_s = torch.empty(n_samples, dtype=torch.float64, device=dev)
    it_s = torch.empty(n_samples, dtype=torch.int32, device=dev)
    for t in range(n_samples):
        api.draw_sample(m, s, seed, t, out=idx)
        C.copy_(C_w)
        desc, _, _ = api.make_desc([s], [k], seed=seed, sample_id=[t], d=d)
        api.lloyd_batch(X, idx, desc, C, max_iter=max_iter, rel_tol=rel_tol, precision=precision,
                        f_out=f_s[t:t + 1], iters_out=it_s[t:t + 1])
        api.keep_best(C, f_s[t:t + 1], C_w, f_hat, k, d)
    labels = counts = sse = None
    if final_assign:
        labels, counts, sse = api.assign_sse(X, C_w, precision=precision)
    return WorkerResult(C_w, f_hat, f_s, it_s, labels, counts, sse)


@dataclass
class StrategyState:
    C_inc: torch.Tensor   # W x k x d incumbents
    f_inc: torch.Tensor   # W float64
    round: int = 0


def new_state(W: int, k: int, d: int, device) -> StrategyState:
    return StrategyState(
        torch.full((W, k, d), float("nan"), dtype=torch.float32, device=device),
        torch.full((W,), float("inf"), dtype=torch.float64, device=device))


def strategy_round(X, state: StrategyState, *, s: int, k: int, seed: int, cooperative: bool,
                   max_iter=300, rel_tol=1e-4, precision=api.PREC_FP32, work=None):
    """One round of W workers as one batched launch.  Worker w processes
    sample id round*W + w.  Competitive: starts from its own incumbent;
    cooperative: from the best incumbent (lowest index on ties).  Returns
    (f, iters) of the round."""
    m, d = X.shape
    W = state.f_inc.numel()
    dev = X.device
    if work is None:
        work = {}
    C = work.get("C")
    if C is None or C.shape != state.C_inc.shape:
        C = work["C"] = torch.empty_like(state.C_inc)
    if cooperative:
        Cb, _, _ = api.select_best(state.C_inc, state.f_inc, k, d)
        C.copy_(Cb.unsqueeze(0).expand(W, k, d))
    else:
        C.copy_(state.C_inc)
    ids = [state.round * W + w for w in range(W)]
    desc, idx_len, _ = api.make_desc([s] * W, [k] * W, seed=seed, sample_id=ids, d=d)
    idx = work.get("idx")
    if idx is None or idx.numel() != idx_len:
        idx = work["idx"] = torch.empty(idx_len, dtype=torch.int64, device=dev)
    api.draw_samples(m, desc, idx_len, out=idx)
    f, it, _ = api.lloyd_batch(X, idx, desc, C, max_iter=max_iter, rel_tol=rel_tol,
                               precision=precision)
    api.keep_best(C, f, state.C_inc, state.f_inc, k, d)
    state.round += 1
    return f, it


def run_strategy(X, *, W: int, s: int, k: int, seed: int, n_rounds: int, strategy: str,
                 n_competitive: int = 0, max_iter=300, rel_tol=1e-4, precision=api.PREC_FP32):
    """HPClust-competitive / -cooperative / -hybrid over n_rounds rounds;
    hybrid runs n_competitive competitive rounds first.  Returns the state,
    the best incumbent and the final assignment."""
    m, d = X.shape
    state = new_state(W, k, d, X.device)
    work = {}
    for r in range(n_rounds):
        coop = strategy == "cooperative" or (strategy == "hybrid" and r >= n_competitive)
        if strategy not in ("competitive", "cooperative", "hybrid"):
            raise ValueError(strategy)
        strategy_round(X, state, s=s, k=k, seed=seed, cooperative=coop, max_iter=max_iter,
                       rel_tol=rel_tol, precision=precision, work=work)
    Cb, fb, wb = api.select_best(state.C_inc, state.f_inc, k, d)
    labels, counts, sse = api.assign_sse(X, Cb, precision=precision)
    return state, Cb, fb, wb, labels, counts, sse


@dataclass
class BudgetLog:
    """Per-round record of a time-budgeted run (times in seconds from the
    start, measured with HIP events on the run's stream)."""
    t_round: list          # end time of each round
    f_best: list           # best sample objective over workers after each round
    n_samples: list        # samples processed so far (n_s)
    n_dist: list           # distance evaluations so far (n_d)
    t: float               # time of the last incumbent update of the best worker
    t_bar: float | None    # time the best objective first reached f_bar (None: never)
    C_best: torch.Tensor   # k x d incumbent of the best worker
    f_hat: float
    sse: float             # full-data objective of C_best
    rounds: int


def run_budget(X, *, W: int, s: int, k: int, seed: int, T: float, strategy: str = "competitive",
               T1: float | None = None, f_bar: float | None = None, max_rounds: int = 100000,
               precision=api.PREC_FP32):
    """HPClust under a time limit (Section 6.5: stop at the CPU time limit T;
    Section 6.4: t, the time until the last solution update, and t_bar, the
    time until any worker reaches the baseline sample objective f_bar).

    Rounds of W workers run until the elapsed time reaches T; hybrid runs
    competitive rounds until T1 (default T / 2, the split of the scaling
    study) and cooperative rounds after.  n_d counts, as the paper's
    appendix does, s per seeded sample's first centre plus 3 s per further
    seeded centre (cold starts), s k per assignment pass, and m k for the
    final assignment; the rare re-seeds of emptied clusters inside a run are
    not counted."""
    import time as _time

    if strategy not in ("competitive", "cooperative", "hybrid"):
        raise ValueError(strategy)
    m, d = X.shape
    T1 = T / 2 if T1 is None else T1
    state = new_state(W, k, d, X.device)
    work = {}
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    torch.cuda.synchronize()
    wall0 = _time.perf_counter()
    log = BudgetLog([], [], [], [], 0.0, None, None, float("inf"), float("inf"), 0)
    n_dist = 0
    f_best_prev = float("inf")
    for r in range(max_rounds):
        elapsed = _time.perf_counter() - wall0
        if elapsed >= T:
            break
        coop = strategy == "cooperative" or (strategy == "hybrid" and elapsed >= T1)
        cold = bool(torch.isnan(state.C_inc[:, 0, 0]).any().item()) if r == 0 else False
        f, it = strategy_round(X, state, s=s, k=k, seed=seed, cooperative=coop,
                               precision=precision, work=work)
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        e.synchronize()
        t_r = e0.elapsed_time(e) / 1e3
        n_dist += int(it.sum().item()) * s * k
        if cold:
            n_dist += W * s * (1 + 3 * (k - 1))
        fb = float(state.f_inc.min().item())
        log.t_round.append(t_r)
        log.f_best.append(fb)
        log.n_samples.append((r + 1) * W)
        log.n_dist.append(n_dist)
        if fb < f_best_prev:
            log.t = t_r
            f_best_prev = fb
        if f_bar is not None and log.t_bar is None and fb <= f_bar:
            log.t_bar = t_r
        log.rounds = r + 1
    Cb, fb, wb = api.select_best(state.C_inc, state.f_inc, k, d)
    _, _, sse = api.assign_sse(X, Cb, want_labels=False, want_counts=False, precision=precision)
    log.C_best, log.f_hat, log.sse = Cb, float(fb.item()), float(sse.item())
    if log.n_dist:
        log.n_dist[-1] += m * k
    return log


@dataclass
class StreamResult:
    state: StrategyState
    f_rounds: list         # per round: f of every worker (host float64 arrays)
    iters_rounds: list     # per round: passes of every worker
    t_rounds: list         # per round: end time in seconds from the start (HIP events)


def run_stream(source, *, W: int, s: int, k: int, d: int, seed: int, n_rounds: int,
               strategy: str = "competitive", n_competitive: int = 0, max_iter=300,
               rel_tol=1e-4, precision=api.PREC_FP32):
    """HPClust on a stream of data (the infinitely tall setting of Section 1,
    m = infinity; streaming sources are the paper's stated future direction):
    round r's samples are the next W*s points of the stream, source(r)
    returning them as a host float32 array of shape (W*s, d), worker w taking
    rows [w*s, (w+1)*s).  Blocks are staged in pinned host memory and copied
    to the device on a second stream while the previous round's kernels run
    (two buffers; events order each round after its copy and each copy after
    the round that last read its buffer).  Incumbents and strategies are as
    in strategy_round; sample ids are r*W + w."""
    import numpy as np

    if strategy not in ("competitive", "cooperative", "hybrid"):
        raise ValueError(strategy)
    dev = torch.device("cuda", torch.cuda.current_device())
    n = W * s
    pinned = [torch.empty((n, d), dtype=torch.float32, pin_memory=True) for _ in range(2)]
    bufs = [torch.empty((n, d), dtype=torch.float32, device=dev) for _ in range(2)]
    copied = [torch.cuda.Event() for _ in range(2)]
    used = [torch.cuda.Event() for _ in range(2)]
    staged = [None, None]  # copy-stream events guarding the pinned buffers
    compute = torch.cuda.current_stream()
    copy_stream = torch.cuda.Stream()
    idx = torch.arange(n, dtype=torch.int64, device=dev)
    state = new_state(W, k, d, dev)
    C = torch.empty_like(state.C_inc)
    t0 = torch.cuda.Event(enable_timing=True)
    t0.record(compute)
    ends = []
    out_f, out_it = [], []

    def stage(r):
        b = r % 2
        if staged[b] is not None:
            staged[b].synchronize()  # the previous copy out of this pinned buffer is done
        block = np.asarray(source(r), dtype=np.float32)
        if block.shape != (n, d):
            raise ValueError(f"source({r}) returned shape {block.shape}, expected {(n, d)}")
        pinned[b].numpy()[...] = block
        with torch.cuda.stream(copy_stream):
            copy_stream.wait_event(used[b])  # the round that last read bufs[b] has finished
            bufs[b].copy_(pinned[b], non_blocking=True)
            copied[b].record(copy_stream)
        staged[b] = torch.cuda.Event()
        staged[b].record(copy_stream)

    for b in range(2):
        used[b].record(compute)
    stage(0)
    for r in range(n_rounds):
        b = r % 2
        coop = strategy == "cooperative" or (strategy == "hybrid" and r >= n_competitive)
        compute.wait_event(copied[b])
        if coop:
            Cb, _, _ = api.select_best(state.C_inc, state.f_inc, k, d)
            C.copy_(Cb.unsqueeze(0).expand(W, k, d))
        else:
            C.copy_(state.C_inc)
        desc, _, _ = api.make_desc([s] * W, [k] * W, seed=seed,
                                   sample_id=[r * W + w for w in range(W)], d=d)
        f, it, _ = api.lloyd_batch(bufs[b], idx, desc, C, max_iter=max_iter, rel_tol=rel_tol,
                                   precision=precision)
        api.keep_best(C, f, state.C_inc, state.f_inc, k, d)
        used[b].record(compute)
        e = torch.cuda.Event(enable_timing=True)
        e.record(compute)
        ends.append(e)
        out_f.append(f)
        out_it.append(it)
        state.round += 1
        if r + 1 < n_rounds:
            stage(r + 1)  # host fill and copy overlap this round's kernels
    torch.cuda.synchronize()
    return StreamResult(state, [f.cpu().numpy() for f in out_f],
                        [i.cpu().numpy() for i in out_it],
                        [t0.elapsed_time(e) / 1e3 for e in ends])
