"""The hot path at the full sizes of its workloads, in the launch
configuration the benchmark uses (plans, autotuned, the round captured in a
HIP graph for the uneven batch).  The oracle checks what it can compute
one by one -- whole samples picked from each batch, the labels of sampled
data rows -- and properties that hold at any size cover the rest.

Workloads (recipes in the synthetic module):
  plain batched  m = 10^7, d = 16, k in {5, 10, 25}, 256 samples of 20,000
  uneven         m = 2*10^7, d = 32, 1,024 samples, s in [1e3, 1e5], k in [2, 50]
  precision      m = 10^8, d = 64, k = 100, 128 samples of 50,000, all three screenings
"""
import numpy as np
import pytest
import torch

import synthetic
from tests.tolerances import F_REL, SSE_REL, assert_centroids, assert_labels, diag_clean, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_2311_04517_amd import api

    api.version()
    return api


def _say(*a):
    print("[fullsize]", *a, flush=True)


def _dn(desc, rows):
    return dict(idx_offset=[desc[b].idx_offset for b in rows], s=[desc[b].s for b in rows],
                k=[desc[b].k for b in rows], c_offset=[desc[b].c_offset for b in rows],
                seed=[desc[b].seed for b in rows], sample_id=[desc[b].sample_id for b in rows])


def _check_samples(orc, X, idx, desc, rows, C_start, Cg, fg, itg, d, m, seed, compared=None):
    """Oracle runs of the chosen samples on their own rows (the sample's
    points in draw order), compared where the oracle reports no decision
    within rounding of its threshold.  Returns the number compared (and
    lists the compared samples in ``compared``)."""
    if compared is None:
        compared = []
    sub_idx, subs, offs = [], [], []
    off = 0
    for b in rows:
        ds = desc[b]
        ii = idx[ds.idx_offset:ds.idx_offset + ds.s].cpu()
        assert np.array_equal(ii.numpy(), orc.draw_sample(m, ds.s, ds.seed, ds.sample_id))
        subs.append(X[ii.cuda()].cpu().numpy())
        offs.append(off)
        off += ds.s
    Xs = np.concatenate(subs)
    dn = _dn(desc, rows)
    co = np.concatenate([[0], np.cumsum([desc[b].k * d for b in rows])[:-1]])
    Co = np.concatenate([C_start[desc[b].c_offset:desc[b].c_offset + desc[b].k * d]
                         for b in rows]).astype(np.float64)
    odesc = dict(idx_offset=offs, s=dn["s"], k=dn["k"], c_offset=co, seed=dn["seed"],
                 sample_id=dn["sample_id"])
    ro = orc.lloyd_batch(Xs, np.arange(len(Xs)), odesc, Co, n_threads=min(16, len(rows)))
    n = 0
    compared.clear()
    for q, b in enumerate(rows):
        ds = desc[b]
        S = Xs[offs[q]:offs[q] + ds.s]
        cg = Cg[ds.c_offset:ds.c_offset + ds.k * d].reshape(ds.k, d)
        assert np.isfinite(cg).all()
        if not diag_clean(ro["diag"][q]):
            continue
        n += 1
        compared.append(b)
        assert itg[b] == ro["iters"][q], (b, itg[b], ro["iters"][q])
        assert rel(fg[b], ro["f"][q]) <= F_REL
        assert_centroids(cg, Co[co[q]:co[q] + ds.k * d].reshape(ds.k, d), S)
    return n


def _check_rows(orc, X, C, labels, n_rows, seed):
    """Labels of sampled data rows against the oracle's argmin."""
    m = X.shape[0]
    rows = torch.from_numpy(np.random.default_rng(seed).choice(m, n_rows, replace=False)).cuda()
    o = orc.assign_sse(X[rows].cpu().numpy(), C.double().cpu().numpy(), want_margins=True)
    assert_labels(labels[rows].cpu().numpy(), o["labels"], o["margins"])


def test_plain_batched_full_size(hp, orc):
    mx = synthetic.plain_batched(device="cuda")
    X = mx.X
    m, d = X.shape
    s, W = 20_000, 256
    Xn_full = None
    for k in (5, 10, 25):
        desc, idx_len, c_len = hp.make_desc([s] * W, [k] * W, seed=2, sample_id=np.arange(W) + 1000 * k,
                                            d=d)
        with hp.Plan(d, desc, idx_len, c_len) as plan:
            idx = torch.empty(idx_len, dtype=torch.int64, device="cuda")
            plan.draw(m, idx)
            C = torch.full((c_len,), float("nan"), device="cuda")
            f, it, _ = plan.lloyd(X, idx, C)
            torch.cuda.synchronize()
            _say(f"plain batched k={k}: passes {it.sum().item()}, mean {it.float().mean().item():.1f}")
            Cg, fg, itg = C.cpu().numpy(), f.cpu().numpy(), it.cpu().numpy()
            assert ((itg >= 1) & (itg <= 300)).all() and np.isfinite(fg).all()
            n = _check_samples(orc, X, idx, desc, [0, 77, 255], np.full(c_len, np.nan), Cg, fg, itg,
                               d, m, 2)
            assert n >= 2
        if k == 25:
            b = int(np.argmin(fg))
            Cb = C[desc[b].c_offset:desc[b].c_offset + k * d].view(k, d).contiguous()
            lab, cnt, sse = hp.assign_sse(X, Cb)
            assert cnt.sum().item() == m
            if Xn_full is None:
                Xn_full = X.cpu().numpy()
            o = orc.assign_sse(Xn_full, Cb.double().cpu().numpy(), want_margins=True)
            assert_labels(lab.cpu().numpy(), o["labels"], o["margins"])
            assert rel(sse.item(), o["sse"]) <= SSE_REL
            _say(f"plain batched full assign: SSE {sse.item():.6e} (oracle {o['sse']:.6e})")


def test_uneven_batch_one_captured_launch(hp, orc, tmp_path):
    from paper_2311_04517_amd import tuning

    mx = synthetic.uneven(device="cuda")
    X = mx.X
    m, d = X.shape
    ss, ks = synthetic.uneven_sizes(1024, seed=3)
    n = len(ss)
    desc, idx_len, c_len = hp.make_desc(ss, ks, seed=3, sample_id=np.arange(n), d=d)
    plan = hp.Plan(d, desc, idx_len, c_len)
    idx = torch.empty(idx_len, dtype=torch.int64, device="cuda")
    C = torch.empty(c_len, device="cuda")
    C_inc = torch.full((c_len,), float("nan"), device="cuda")
    f_inc = torch.full((n,), float("inf"), dtype=torch.float64, device="cuda")
    f_out = torch.empty(n, dtype=torch.float64, device="cuda")
    it_out = torch.empty(n, dtype=torch.int32, device="cuda")
    # autotune on warm passes of a throwaway draw, then restore the ids
    plan.draw(m, idx)
    Ct = torch.full((c_len,), float("nan"), device="cuda")
    plan.lloyd(X, idx, Ct, max_iter=2)
    cfg, ms = tuning.tuned(plan, X, idx, Ct, path=str(tmp_path / "t.json"), max_iter=2)
    _say(f"uneven: autotuned {cfg} ({ms:.2f} ms)")
    del Ct
    plan.capture_round(X, idx, C, C_inc, f_inc, f_out, it_out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    plan.replay(1)
    e1.record()
    torch.cuda.synchronize()
    _say(f"uneven: one cold round of {n} samples (sum s {int(ss.sum())}) in "
         f"{e0.elapsed_time(e1):.1f} ms, passes {it_out.sum().item()}")
    fg, itg, Cg = f_out.cpu().numpy(), it_out.cpu().numpy(), C.cpu().numpy()
    assert ((itg >= 1) & (itg <= 300)).all() and np.isfinite(fg).all() and np.isfinite(Cg).all()
    assert torch.equal(f_inc, f_out)  # first round: every sample becomes its worker's incumbent
    # the six smallest, the median and the two largest samples by work s*k
    # (the largest, s near 1e5 and k near 50, set the length of the batch)
    work = ss * ks
    srt = np.argsort(work)
    largest = [int(i) for i in srt[-2:]]
    pick = [int(i) for i in srt[:6]] + [int(srt[n // 2])] + largest
    _say(f"uneven: comparing samples {pick} (s, k of the largest: "
         f"{[(int(ss[i]), int(ks[i])) for i in largest]})")
    done = []
    nc = _check_samples(orc, X, idx, desc, pick, np.full(c_len, np.nan), Cg, fg, itg, d, m, 3,
                        compared=done)
    _say(f"uneven: {nc} of {len(pick)} samples compared with the oracle")
    assert nc >= 7
    assert any(b in done for b in largest), "neither of the largest samples was compared"
    plan.close()


@pytest.fixture(scope="module")
def precision_data():
    mx = synthetic.precision_set(device="cuda")
    X = mx.X
    del mx
    _say(f"precision set generated: {tuple(X.shape)}")
    yield X
    del X
    torch.cuda.empty_cache()


PREC_RUNS = {}


@pytest.mark.parametrize("prec", [2, 1, 0])
def test_precision_set_lloyd_full_size(hp, orc, precision_data, prec):
    """A cold batch of the precision workload (128 samples of 50,000, k =
    100, d = 64) in each screening (BF16x3 first: the workload's default):
    both sampled workers against the oracle, and identical pass counts,
    objectives and centroids across the screenings."""
    X = precision_data
    m, d = X.shape
    s, k, W = 50_000, 100, 128
    desc, idx_len, c_len = hp.make_desc([s] * W, [k] * W, seed=4, sample_id=np.arange(W), d=d)
    with hp.Plan(d, desc, idx_len, c_len, precision=prec) as plan:
        idx = torch.empty(idx_len, dtype=torch.int64, device="cuda")
        plan.draw(m, idx)
        C = torch.full((c_len,), float("nan"), device="cuda")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        f, it, _ = plan.lloyd(X, idx, C)
        e1.record()
        torch.cuda.synchronize()
        _say(f"precision {prec}: cold batch in {e0.elapsed_time(e1):.1f} ms, "
             f"passes {it.sum().item()}")
        Cg, fg, itg = C.cpu().numpy(), f.cpu().numpy(), it.cpu().numpy()
        assert ((itg >= 1) & (itg <= 300)).all() and np.isfinite(fg).all()
        nc = _check_samples(orc, X, idx, desc, [0, 101], np.full(c_len, np.nan), Cg, fg, itg, d,
                            m, 4)
        _say(f"precision {prec}: {nc} of 2 samples compared with the oracle")
        assert nc == 2
    PREC_RUNS[prec] = (Cg, fg, itg)
    for other, (Co, fo, ito) in PREC_RUNS.items():
        # every screening decides in FP64: same passes; objectives and
        # centroids agree up to the order of the FP64 sums
        assert np.array_equal(itg, ito), (prec, other)
        assert np.allclose(fg, fo, rtol=1e-11, atol=0)
        assert np.allclose(Cg, Co, rtol=1e-6, atol=1e-5)


def test_precision_set_assign_full_size(hp, orc, precision_data):
    X = precision_data
    m, d = X.shape
    k = 100
    assert PREC_RUNS, "runs after the Lloyd test"
    Cg, fg, _ = next(iter(PREC_RUNS.values()))
    b = int(np.argmin(fg))
    Cb = torch.from_numpy(Cg[b * k * d:(b + 1) * k * d].reshape(k, d).copy()).cuda()
    lab16, cnt16, sse16 = hp.assign_sse(X, Cb, precision=hp.PREC_BF16_MFMA)
    lab32, cnt32, sse32 = hp.assign_sse(X, Cb, precision=hp.PREC_FP32)
    lab3, cnt3, sse3 = hp.assign_sse(X, Cb, precision=hp.PREC_BF16X3_MFMA)
    # every screening takes each decision in FP64: identical labels, counts
    # and (same launch shape and summation order) identical SSE
    assert torch.equal(lab16, lab32) and torch.equal(cnt16, cnt32)
    assert torch.equal(lab3, lab32) and torch.equal(cnt3, cnt32)
    assert sse16.item() == sse32.item() == sse3.item()
    assert cnt16.sum().item() == m
    _check_rows(orc, X, Cb, lab3, 200_000, seed=4)
    _say(f"precision: full assign SSE {sse3.item():.6e}")


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_metric_workload_full_size(hp, orc, tmp_path, prec):
    """The benchmark's own configuration: m = 1e7, d = 32, k = 25, 1,024
    workers x s = 10,000, autotuned plan, a cold round then a warm round
    from the incumbents; sampled workers of both rounds against the oracle,
    and the full assignment of the best incumbent on sampled rows."""
    from paper_2311_04517_amd import tuning

    mx = synthetic.metric_set(device="cuda")
    X = mx.X
    m, d = X.shape
    W, s, k = 1024, 10_000, 25
    desc, idx_len, c_len = hp.make_desc([s] * W, [k] * W, seed=1, sample_id=np.arange(W), d=d)
    plan = hp.Plan(d, desc, idx_len, c_len, precision=prec)
    idx = torch.empty(idx_len, dtype=torch.int64, device="cuda")
    plan.draw(m, idx)
    Ct = torch.full((c_len,), float("nan"), device="cuda")
    plan.lloyd(X, idx, Ct)
    tuning.tuned(plan, X, idx, Ct, path=str(tmp_path / "t.json"), max_iter=3)
    del Ct
    C = torch.empty(c_len, device="cuda")
    C_inc = torch.full((c_len,), float("nan"), device="cuda")
    f_inc = torch.full((W,), float("inf"), dtype=torch.float64, device="cuda")
    f_out = torch.empty(W, dtype=torch.float64, device="cuda")
    it_out = torch.empty(W, dtype=torch.int32, device="cuda")
    for r in range(2):
        start = C_inc.cpu().numpy()
        plan.round(X, idx, C, C_inc, f_inc, f_out, it_out)
        torch.cuda.synchronize()
        fg, itg, Cg = f_out.cpu().numpy(), it_out.cpu().numpy(), C.cpu().numpy()
        _say(f"metric workload prec {prec} round {r}: passes {itg.sum()}")
        assert ((itg >= 1) & (itg <= 300)).all() and np.isfinite(Cg).all()
        rdesc, _, _ = hp.make_desc([s] * W, [k] * W, seed=1, sample_id=np.arange(W) + r * W, d=d)
        nc = _check_samples(orc, X, idx, rdesc, [0, 511, 1023], start, Cg, fg, itg, d, m, 1)
        assert nc >= 2
    Cb, fb, wb = hp.select_best(C_inc.view(W, k, d), f_inc, k, d)
    lab, cnt, sse = hp.assign_sse(X, Cb, precision=prec)
    assert cnt.sum().item() == m
    _check_rows(orc, X, Cb, lab, 200_000, seed=5)
    plan.close()
