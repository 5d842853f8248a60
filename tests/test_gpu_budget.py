"""The time-budgeted driver (Section 6.5 time limit; Section 6.4 metrics t,
t_bar, n_d, n_s) on the GPU: its bookkeeping against the oracle's
single-worker loop, and a timed hybrid run on the scaling study's data."""
import numpy as np
import pytest
import torch

import synthetic
from tests.tolerances import F_REL, SSE_REL, diag_clean, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_2311_04517_amd import api

    api.version()
    return api


def test_budget_counts_match_oracle_worker_loop(hp, orc):
    """One worker, a fixed number of rounds: the incumbent's f, the samples
    processed, and n_d equal the oracle's single-worker loop (whose counter
    follows the paper's appendix), where no re-seed happened after the cold
    start."""
    from paper_2311_04517_amd import driver

    mx = synthetic.plain_small()
    Xn, Xg = mx.X.numpy(), mx.X.cuda()
    s, k, N = 2000, 10, 6
    checked = 0
    for seed in range(3):
        log = driver.run_budget(Xg, W=1, s=s, k=k, seed=seed, T=1e9, max_rounds=N)
        wo = orc.worker_loop(Xn, s=s, k=k, n_samples=N, seed=seed)
        assert log.rounds == N and log.n_samples == list(range(1, N + 1))
        assert all(b <= a for a, b in zip(log.f_best, log.f_best[1:]))
        assert all(b >= a for a, b in zip(log.t_round, log.t_round[1:]))
        if not diag_clean(wo["diag"]):
            continue
        checked += 1
        assert rel(log.f_hat, wo["f_hat"]) <= F_REL
        assert rel(log.sse, wo["sse"]) <= SSE_REL
        if wo["diag"]["n_seeded_rows"] == k:
            assert log.n_dist[-1] == wo["diag"]["n_dist"]
    assert checked >= 2, f"only {checked} of 3 seeds compared"


def test_budget_hybrid_on_scaling_data(hp):
    """Hybrid (T1 = T2 = T/2) on the scaling study's data, i = 2: the run
    stops once T has elapsed, switches to cooperative rounds after T1, and
    its records are consistent."""
    from paper_2311_04517_amd import driver

    mx = synthetic.scaling_blobs(2, seed=1, device="cuda")
    m = mx.X.shape[0]
    s = synthetic.scaling_sample_size(3 ** 9)
    T = 0.4
    log = driver.run_budget(mx.X, W=64, s=s, k=10, seed=1, T=T, strategy="hybrid")
    assert log.rounds >= 2
    assert log.t_round[-2] < T + 0.5  # the last round started before T
    assert all(b <= a for a, b in zip(log.f_best, log.f_best[1:]))
    assert log.t in log.t_round and log.f_best[log.t_round.index(log.t)] == log.f_best[-1]
    assert log.n_samples[-1] == 64 * log.rounds
    assert np.isfinite(log.sse) and log.sse > 0
    # t_bar: the first round whose best sample objective reached f_bar
    f_bar = log.f_best[len(log.f_best) // 2]
    log2 = driver.run_budget(mx.X, W=64, s=s, k=10, seed=1, T=T, strategy="hybrid", f_bar=f_bar,
                             max_rounds=log.rounds)
    assert log2.t_bar is not None and log2.t_bar <= log2.t_round[-1]
