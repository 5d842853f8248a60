"""Batch plans on the GPU: uneven samples in one persistent launch under
every launch configuration, the worker-loop round captured in a HIP graph
and replayed, and the autotuner -- all against the FP64 oracle and against
the one-shot entry points."""
import numpy as np
import pytest
import torch

import synthetic
from tests.tolerances import F_REL, assert_centroids, assert_labels, diag_clean, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_2311_04517_amd import api

    api.version()
    return api


def _uneven(hp, orc, n, d, seed, m=60_000, s_lo=100, s_hi=5000, k_hi=30):
    mx = synthetic.gaussian_mixture(m, d, 14, seed=seed, centre_box=12.0)
    Xn = mx.X.numpy()
    rng = np.random.default_rng(seed)
    ss = rng.integers(s_lo, s_hi, size=n)
    ks = np.minimum(rng.integers(2, k_hi, size=n), ss)
    sid0 = 1000 * seed
    desc, idx_len, c_len = hp.make_desc(ss, ks, seed=seed, sample_id=np.arange(n) + sid0, d=d)
    return Xn, mx.X.cuda(), desc, idx_len, c_len, ss, ks, sid0


def _dn(desc):
    n = len(desc)
    return dict(idx_offset=[desc[b].idx_offset for b in range(n)], s=[desc[b].s for b in range(n)],
                k=[desc[b].k for b in range(n)], c_offset=[desc[b].c_offset for b in range(n)],
                seed=[desc[b].seed for b in range(n)],
                sample_id=[desc[b].sample_id for b in range(n)])


CONFIGS = [dict(), dict(wg_per_cu=1, copies=1, order=0), dict(wg_per_cu=2, copies=4, order=1),
           dict(wg_per_cu=0, copies=2, order=1)]



@pytest.mark.parametrize("prec", [0, 2])
@pytest.mark.parametrize("d,n,s,parts", [(32, 40, 8192, 8), (64, 24, 16384, 16), (64, 30, 4096, 4)])
def test_plan_parts_beyond_the_resident_grid(hp, orc, prec, d, n, s, parts):
    """More samples x parts than resident workgroups (one per CU): the
    samples run in turn, each on `parts` workgroups, later ones from the
    queue as earlier ones finish; two samples start with a centroid far from
    every point, reseed in the first pass and finish alone (their other
    parts take queued tasks early).  Every configuration gives the pass
    counts and labels of the automatic one and of the oracle."""
    m, k = 100_000, 12
    mx = synthetic.gaussian_mixture(m, d, k, seed=90 + d, centre_box=10.0, std=1.0)
    Xn, centres = mx.X.numpy(), mx.centres.numpy()
    rng = np.random.default_rng(d + n)
    C0 = np.stack([centres + rng.normal(0, 0.6, (k, d)) for _ in range(n)]).astype(np.float32)
    C0[3, 5] = 1e4
    C0[n - 2, 0] = -1e4
    Xg = mx.X.cuda()
    desc, idx_len, c_len = hp.make_desc([s] * n, [k] * n, seed=9, sample_id=np.arange(n), d=d)
    idx = hp.draw_samples(m, desc, idx_len)
    idx_n = idx.cpu().numpy()
    outs = []
    with hp.Plan(d, desc, idx_len, c_len, precision=prec) as plan:
        for cfg in (dict(), dict(wg_per_cu=1, parts=parts), dict(wg_per_cu=1, parts=2, copies=1)):
            plan.set_tune(**cfg)
            assert plan.tune.parts == cfg.get("parts", 0)
            C = torch.from_numpy(C0.ravel().copy()).cuda()
            f, it, lab = plan.lloyd(Xg, idx, C, want_labels=True)
            outs.append((C.cpu().numpy(), f.cpu().numpy(), it.cpu().numpy(), lab.cpu().numpy()))
    (Cg, fg, itg, lg) = outs[0]
    assert np.isfinite(fg).all() and (itg > 0).all()
    ros = [orc.lloyd(Xn, idx_n[b * s:(b + 1) * s], k, C0[b].astype(np.float64), seed=9,
                     sample_id=b, want_margins=True) for b in range(n)]
    # configurations differ only in the order the partial sums are added (the
    # LDS sums in no fixed order): on samples where no decision of the
    # oracle's run sits within rounding of its threshold they take the same
    # decisions (labels may differ only at points within rounding of a tie);
    # elsewhere a reseed draw or a stop test may go either way
    clean = [b for b in range(n) if diag_clean(ros[b].diag)]
    assert len(clean) >= n // 2
    for Co, fo, ito, lo in outs[1:]:
        for b in clean:
            sl, cl = slice(b * s, (b + 1) * s), slice(b * k * d, (b + 1) * k * d)
            assert itg[b] == ito[b], (b, itg[b], ito[b])
            assert_labels(lo[sl], lg[sl], ros[b].margins, what=f"sample {b} across configurations")
            assert np.allclose(fg[b], fo[b], rtol=1e-11, atol=0)
            assert np.allclose(Cg[cl], Co[cl], rtol=1e-6, atol=1e-6)
    checked = 0
    for b in range(n):
        ib = idx_n[b * s:(b + 1) * s]
        ro = ros[b]
        if b in (3, n - 2):
            assert ro.diag["n_seed_calls"] >= 1
        if not diag_clean(ro.diag):
            continue
        checked += 1
        for Co, fo, ito, lo in outs:
            assert ito[b] == ro.iters and rel(fo[b], ro.f) <= F_REL, (b, ito[b], ro.iters)
            assert_centroids(Co[b * k * d:(b + 1) * k * d].reshape(k, d), ro.C, Xn[ib])
            assert_labels(lo[b * s:(b + 1) * s], ro.labels, ro.margins)
    assert checked >= n // 2

@pytest.mark.parametrize("prec", [0, 1, 2])
def test_plan_lloyd_every_config_matches_oracle(hp, orc, prec):
    n, d = 40, 32
    Xn, Xg, desc, idx_len, c_len, ss, ks, sid0 = _uneven(hp, orc, n, d, seed=3)
    dn = _dn(desc)
    idx = hp.draw_samples(Xn.shape[0], desc, idx_len)
    idx_n = idx.cpu().numpy()
    C0 = np.full(c_len, np.nan)
    Co = C0.copy()
    ro = orc.lloyd_batch(Xn, idx_n, dn, Co, n_threads=8)
    clean = [b for b in range(n) if diag_clean(ro["diag"][b])]
    assert len(clean) >= n // 2
    ref = None
    with hp.Plan(d, desc, idx_len, c_len, precision=prec) as plan:
        for cfg in CONFIGS:
            if cfg:
                plan.set_tune(**cfg)
            C = torch.full((c_len,), float("nan"), device="cuda")
            f, it, _ = plan.lloyd(Xg, idx, C)
            Cg, fg, itg = C.cpu().numpy(), f.cpu().numpy(), it.cpu().numpy()
            for b in clean:
                io, s, k, co = dn["idx_offset"][b], dn["s"][b], dn["k"][b], dn["c_offset"][b]
                assert itg[b] == ro["iters"][b], (cfg, b)
                assert rel(fg[b], ro["f"][b]) <= F_REL
                assert_centroids(Cg[co:co + k * d].reshape(k, d),
                                 Co[co:co + k * d].reshape(k, d), Xn[idx_n[io:io + s]])
            if ref is None:
                # the one-shot entry point gives the same results
                C1 = torch.full((c_len,), float("nan"), device="cuda")
                f1, it1, _ = hp.lloyd_batch(Xg, idx, desc, C1, precision=prec)
                assert torch.equal(it1, it) and torch.equal(f1, f) and torch.equal(C1, C)
                ref = (itg, fg)
            else:
                for b in clean:
                    assert itg[b] == ref[0][b] and rel(fg[b], ref[1][b]) <= 1e-12


@pytest.mark.parametrize("d", [16, 64])
def test_plan_round_graph_replays_match_eager_and_oracle(hp, orc, d):
    """One worker-loop round (draw, start from incumbent, Lloyd, keep-best,
    advance sample ids) captured once and replayed round after round, with
    the program's own work and synchronisations in between: every replay
    equals the same round run eagerly, and each round equals the oracle
    started from the incumbents the GPU held before it.  At d = 64 the warm
    rounds share their samples between two workgroups (the captured
    sequence zeroes the exchange flags with a fill kernel)."""
    n, rounds = 24, 4
    Xn, Xg, desc, idx_len, c_len, ss, ks, sid0 = _uneven(hp, orc, n, d, seed=5, s_hi=3000)
    dn = _dn(desc)
    m = Xn.shape[0]

    def bufs():
        return dict(idx=torch.empty(idx_len, dtype=torch.int64, device="cuda"),
                    C=torch.empty(c_len, device="cuda"),
                    C_inc=torch.full((c_len,), float("nan"), device="cuda"),
                    f_inc=torch.full((n,), float("inf"), dtype=torch.float64, device="cuda"),
                    f_out=torch.empty(n, dtype=torch.float64, device="cuda"),
                    iters_out=torch.empty(n, dtype=torch.int32, device="cuda"))

    E, G = bufs(), bufs()
    pe = hp.Plan(d, desc, idx_len, c_len)
    pg = hp.Plan(d, desc, idx_len, c_len)
    pg.capture_round(Xg, G["idx"], G["C"], G["C_inc"], G["f_inc"], G["f_out"], G["iters_out"])
    n_checked = 0
    for r in range(rounds):
        start = E["C_inc"].double().cpu().numpy()
        f_before = E["f_inc"].cpu().numpy()
        pe.round(Xg, E["idx"], E["C"], E["C_inc"], E["f_inc"], E["f_out"], E["iters_out"])
        junk = torch.randn(1 << 20, device="cuda")
        junk.mul_(2.0).sum().item()  # the program's own eager work between replays
        pg.replay(1)
        torch.cuda.synchronize()
        for key in ("idx", "C", "C_inc", "f_inc", "f_out", "iters_out"):
            assert torch.equal(E[key], G[key]), (r, key)
        idx_n = E["idx"].cpu().numpy()
        ref_idx = np.concatenate([orc.draw_sample(m, int(s), 5, sid0 + r * n + b)
                                  for b, s in enumerate(ss)])
        assert np.array_equal(idx_n, ref_idx)
        dr = dict(dn, sample_id=[sid0 + r * n + b for b in range(n)])
        Co = start.copy()
        ro = orc.lloyd_batch(Xn, idx_n, dr, Co, n_threads=8)
        fo, ito = E["f_out"].cpu().numpy(), E["iters_out"].cpu().numpy()
        f_inc = E["f_inc"].cpu().numpy()
        for b in range(n):
            assert f_inc[b] == min(f_before[b], fo[b])
            if not diag_clean(ro["diag"][b]):
                continue
            n_checked += 1
            assert ito[b] == ro["iters"][b]
            assert rel(fo[b], ro["f"][b]) <= F_REL
    assert n_checked >= rounds * n // 2
    pe.close()
    pg.close()


def test_plan_reset_ids_repeats_the_round(hp):
    n, d = 8, 8
    mx = synthetic.gaussian_mixture(20_000, d, 5, seed=2, centre_box=10.0)
    Xg = mx.X.cuda()
    desc, idx_len, c_len = hp.make_desc([800] * n, [5] * n, seed=2, sample_id=np.arange(n), d=d)
    with hp.Plan(d, desc, idx_len, c_len) as plan:
        outs = []
        for _ in range(2):
            idx = torch.empty(idx_len, dtype=torch.int64, device="cuda")
            C = torch.empty(c_len, device="cuda")
            Ci = torch.full((c_len,), float("nan"), device="cuda")
            fi = torch.full((n,), float("inf"), dtype=torch.float64, device="cuda")
            fo = torch.empty(n, dtype=torch.float64, device="cuda")
            io = torch.empty(n, dtype=torch.int32, device="cuda")
            plan.round(Xg, idx, C, Ci, fi, fo, io)
            outs.append((idx, Ci, fi))
            plan.reset_ids()
        for a, b in zip(*outs):
            assert torch.equal(a, b)


def test_autotune_keeps_results(hp, orc, tmp_path):
    from paper_2311_04517_amd import tuning

    n, d, s, k = 96, 32, 4000, 25
    mx = synthetic.gaussian_mixture(200_000, d, 25, seed=7, centre_box=20.0, std=2.0)
    Xg = mx.X.cuda()
    desc, idx_len, c_len = hp.make_desc([s] * n, [k] * n, seed=7, sample_id=np.arange(n), d=d)
    idx = hp.draw_samples(200_000, desc, idx_len)
    with hp.Plan(d, desc, idx_len, c_len) as plan:
        C = torch.full((c_len,), float("nan"), device="cuda")
        f0, it0, _ = plan.lloyd(Xg, idx, C)  # default configuration
        Cw = C.clone()
        path = str(tmp_path / "tune.json")
        cfg, ms = tuning.tuned(plan, Xg, idx, Cw, path=path, max_iter=2)
        assert ms is not None and ms > 0
        assert cfg["copies"] in (1, 2, 4) and cfg["wg_per_cu"] >= 1 and cfg["order"] == 0
        assert torch.equal(Cw, C)  # tuning does not touch the caller's centroids
        t = plan.tune
        assert (t.wg_per_cu, t.copies, t.order) == (cfg["wg_per_cu"], cfg["copies"], cfg["order"])
        C2 = torch.full((c_len,), float("nan"), device="cuda")
        f1, it1, _ = plan.lloyd(Xg, idx, C2)
        assert torch.equal(it0, it1)
        assert (torch.abs(f1 - f0) <= 1e-12 * f0).all()
        cfg2, ms2 = tuning.tuned(plan, Xg, idx, Cw, path=path)
        assert ms2 is None and cfg2 == cfg  # served from the cache
