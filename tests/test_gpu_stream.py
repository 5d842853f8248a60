"""Streaming sample source (driver.run_stream): rounds whose samples are the
next points of a host stream, copied on a second stream while the previous
round computes.  The results must equal the same rounds run on the
concatenated data resident on the device (same kernels, seeds and points),
and a streamed worker's sample must match the oracle."""
import numpy as np
import pytest
import torch

import synthetic
from tests.tolerances import F_REL, diag_clean, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_2311_04517_amd import api

    api.version()
    return api


@pytest.mark.parametrize("strategy", ["competitive", "hybrid"])
def test_stream_equals_resident_rounds(hp, orc, strategy):
    from paper_2311_04517_amd import driver

    W, s, k, d, R, seed = 32, 1500, 8, 16, 5, 3
    mx = synthetic.gaussian_mixture(W * s * R, d, 8, seed=9, centre_box=15.0, std=1.5)
    Xn = mx.X.numpy()
    res = driver.run_stream(lambda r: Xn[r * W * s:(r + 1) * W * s], W=W, s=s, k=k, d=d,
                            seed=seed, n_rounds=R, strategy=strategy, n_competitive=2)
    # the same rounds with every block resident on the device
    Xg = mx.X.cuda()
    state = driver.new_state(W, k, d, "cuda")
    C = torch.empty_like(state.C_inc)
    for r in range(R):
        coop = strategy == "hybrid" and r >= 2
        if coop:
            Cb, _, _ = hp.select_best(state.C_inc, state.f_inc, k, d)
            C.copy_(Cb.unsqueeze(0).expand(W, k, d))
        else:
            C.copy_(state.C_inc)
        desc, _, _ = hp.make_desc([s] * W, [k] * W, seed=seed,
                                  sample_id=[r * W + w for w in range(W)], d=d)
        idx = torch.arange(r * W * s, (r + 1) * W * s, dtype=torch.int64, device="cuda")
        f, it, _ = hp.lloyd_batch(Xg, idx, desc, C)
        hp.keep_best(C, f, state.C_inc, state.f_inc, k, d)
        # the FP64 sums take LDS atomics in whatever order the waves
        # arrive, so two runs agree to summation-order rounding, not bits
        assert np.array_equal(it.cpu().numpy(), res.iters_rounds[r])
        assert np.allclose(f.cpu().numpy(), res.f_rounds[r], rtol=1e-12, atol=0)
    assert torch.allclose(state.C_inc, res.state.C_inc, rtol=1e-6, atol=1e-6)
    assert torch.allclose(state.f_inc, res.state.f_inc, rtol=1e-12, atol=0)
    assert all(b >= a for a, b in zip(res.t_rounds, res.t_rounds[1:]))
    # streamed cold samples against the oracle
    checked = 0
    for w in (0, 5, 17, 31):
        S = Xn[w * s:(w + 1) * s]
        ro = orc.lloyd(S, np.arange(s), k, seed=seed, sample_id=w)
        if not diag_clean(ro.diag):
            continue
        checked += 1
        assert res.iters_rounds[0][w] == ro.iters
        assert rel(res.f_rounds[0][w], ro.f) <= F_REL
    assert checked >= 3, f"only {checked} of 4 streamed samples compared"
