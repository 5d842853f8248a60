"""The learned initializer on the GPU against the FP64 set-encoder oracle:
proposals, loss and every parameter gradient (the kernels use BF16 weights
and BF16 activations as matrix-core operands, so the bar is 2e-2 relative),
the Adam update, the proposal-or-K-means++ choice, and training that
improves the proposals."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import setenc as ose
from tests.tolerances import F_REL, diag_clean, rel

pytestmark = pytest.mark.gpu

ENC_REL = 2e-2


@pytest.fixture(scope="module")
def hp():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_2311_04517_amd import api

    api.version()
    return api


def _family(hp, n_sets, s, d, k, seed, template=False):
    X, _ = synthetic.mixture_family(n_sets, s, d=d, n_comp=k, seed=seed, template=template,
                                    device="cuda")
    desc, idx_len, c_len = hp.make_desc([s] * n_sets, [k] * n_sets, seed=seed,
                                        sample_id=np.arange(n_sets), d=d)
    idx = torch.arange(n_sets * s, dtype=torch.int64, device="cuda")
    return X, idx, desc, idx_len, c_len


def _nrel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _to64(params):
    return {n: np.asarray(v, dtype=np.float64) for n, v in params.items()}


@pytest.mark.parametrize("d,k,n_enc,s", [(32, 25, 1024, 3000), (32, 25, 300, 3000),
                                         (7, 5, 512, 200), (32, 3, 16, 40)])
def test_proposals_match_oracle(hp, d, k, n_enc, s):
    """Ragged encoder subsets (n_enc not a multiple of the chunk, s < n_enc)
    and d below the padded width."""
    n = 6
    X, idx, desc, idx_len, c_len = _family(hp, n, s, d, k, seed=d + k)
    model = hp.SetEncoder(d, k, n_enc=n_enc, max_batch=8, seed=3)
    C = torch.empty(c_len, device="cuda")
    model.propose(X, idx, desc, C)
    p64 = _to64(model.get_params(rounded=True))
    Xn = X.cpu().numpy()
    Cg = C.cpu().numpy()
    nb = min(n_enc, s)
    for b in range(n):
        S = Xn[b * s: b * s + nb]
        P = ose.propose(p64, S, k)
        mu, sigma, _ = ose.normalise(S)
        Pg = Cg[b * k * d:(b + 1) * k * d].reshape(k, d)
        assert _nrel((Pg - mu) / sigma, (P - mu) / sigma) <= ENC_REL


def test_loss_and_gradients_match_oracle(hp):
    d, k, n_enc, s, B = 32, 25, 300, 700, 5
    X, idx, desc, idx_len, c_len = _family(hp, B, s, d, k, seed=11)
    Xn = X.cpu().numpy()
    rng = np.random.default_rng(0)
    Tn = np.concatenate([Xn[b * s + rng.choice(s, k, replace=False)] for b in range(B)])
    T = torch.from_numpy(Tn.ravel().copy()).cuda()
    model = hp.SetEncoder(d, k, n_enc=n_enc, max_batch=8, seed=5)
    # a few steps first, so the head is not at its near-zero initial scale
    for _ in range(3):
        model.grad(X, idx, desc, T)
        model.adam(1e-2)
    loss = model.grad(X, idx, desc, T).item()
    gg = model.get_grads()
    p64 = _to64(model.get_params(rounded=True))
    sets = [Xn[b * s: b * s + n_enc] for b in range(B)]
    targets = [Tn[b * k:(b + 1) * k] for b in range(B)]
    lo, go = ose.loss_and_grads(p64, sets, targets, k)
    assert rel(loss, lo) <= ENC_REL
    for name in ose.PARAM_NAMES:
        assert _nrel(gg[name], go[name]) <= ENC_REL, (name, _nrel(gg[name], go[name]))


def test_adam_step(hp):
    d, k, s, B = 8, 4, 200, 3
    X, idx, desc, idx_len, c_len = _family(hp, B, s, d, k, seed=2)
    T = torch.from_numpy(X.cpu().numpy()[:k * B].ravel().copy()).cuda()
    model = hp.SetEncoder(d, k, n_enc=64, max_batch=4, seed=1)
    p0 = model.get_params()
    model.grad(X, idx, desc, T)
    g = model.get_grads()
    model.adam(1e-3)
    p1 = model.get_params()
    for name in ose.PARAM_NAMES:
        gd = g[name].astype(np.float64)
        mhat = 0.1 * gd / (1 - 0.9)
        vhat = 0.001 * gd * gd / (1 - 0.999)
        expect = p0[name] - 1e-3 * mhat / (np.sqrt(vhat) + 1e-8)
        assert np.allclose(p1[name], expect, rtol=1e-5, atol=1e-7), name


def test_learned_seed_falls_back_to_kmeanspp(hp, orc):
    """An untrained encoder's proposals lose to K-means++ on a mixture
    family: the batch then gets exactly the cold start's seeding, and Lloyd
    from it is the cold start's run."""
    d, k, s, n = 16, 10, 2000, 12
    X, idx, desc, idx_len, c_len = _family(hp, n, s, d, k, seed=21)
    model = hp.SetEncoder(d, k, n_enc=512, max_batch=4, seed=9)
    P = model.propose(X, idx, desc, torch.empty(c_len, device="cuda")).cpu().numpy()
    C = torch.empty(c_len, device="cuda")
    C, C_kpp, fp, fk, acc = model.learned_seed(X, idx, desc, C)
    a = acc.cpu().numpy()
    fpn, fkn = fp.cpu().numpy(), fk.cpu().numpy()
    assert np.array_equal(a, (fpn <= fkn).astype(np.int32))
    assert (a == 0).sum() >= n - 1
    Xn = X.cpu().numpy()
    Cg, Ck = C.cpu().numpy(), C_kpp.cpu().numpy()
    idx_n = idx.cpu().numpy()
    for b in range(n):
        blk = slice(b * k * d, (b + 1) * k * d)
        S = Xn[b * s:(b + 1) * s]
        assert rel(fpn[b], ose.sample_objective(S, P[blk].reshape(k, d))) <= F_REL
        assert rel(fkn[b], ose.sample_objective(S, Ck[blk].reshape(k, d))) <= F_REL
        assert np.array_equal(Cg[blk], P[blk] if a[b] else Ck[blk])
        # the seeding is the cold start's: one oracle pass from all-NaN rows
        ro = orc.lloyd(Xn, idx_n[b * s:(b + 1) * s], k, seed=21, sample_id=b, max_iter=1)
        if diag_clean(ro.diag):
            assert np.array_equal(Ck[blk].reshape(k, d), ro.C.astype(np.float32))
    # Lloyd from the chosen seeds is the cold start's run where K-means++ won
    Cl = C.clone()
    f1, it1, _ = hp.lloyd_batch(X, idx, desc, Cl)
    Cc = torch.full((c_len,), float("nan"), device="cuda")
    f2, it2, _ = hp.lloyd_batch(X, idx, desc, Cc)
    for b in range(n):
        if not a[b]:
            blk = slice(b * k * d, (b + 1) * k * d)
            assert it1[b].item() == it2[b].item() and f1[b].item() == f2[b].item()
            assert torch.equal(Cl[blk], Cc[blk])


def test_training_improves_proposals_and_cuts_passes(hp):
    """Trained on method-generated pairs of a family whose normalised
    structure repeats, the encoder's proposals beat the K-means++ seeding on
    held-out samples, are accepted, and Lloyd from them needs fewer passes
    than from the seeding."""
    from paper_2311_04517_amd import learned

    d, k, s = 32, 25, 2000
    n_train, n_test = 768, 64
    X, idx, desc, idx_len, c_len = _family(hp, n_train, s, d, k, seed=31, template=True)
    T, _, _ = learned.method_targets(X, idx, desc, c_len)
    model = hp.SetEncoder(d, k, n_enc=512, max_batch=32, seed=4)
    Xt, idxt, desct, _, c_lent = _family(hp, n_test, s, d, k, seed=37, template=True)
    Tt, _, _ = learned.method_targets(Xt, idxt, desct, c_lent)
    before = learned.heldout_loss(model, Xt, idxt, desct, Tt, batch=32)
    losses = learned.train(model, X, idx, desc, T, steps=400, batch=32, lr=2e-3, lr_final=2e-4)
    after = learned.heldout_loss(model, Xt, idxt, desct, Tt, batch=32)
    assert np.isfinite(losses).all() and after < 0.25 * before
    C = torch.empty(c_lent, device="cuda")
    C, C_kpp, fp, fk, acc = model.learned_seed(Xt, idxt, desct, C)
    assert acc.float().mean().item() >= 0.75
    f_l, it_l, _ = hp.lloyd_batch(Xt, idxt, desct, C.clone())
    f_k, it_k, _ = hp.lloyd_batch(Xt, idxt, desct, C_kpp.clone())
    assert it_l.float().mean().item() < it_k.float().mean().item()
    assert (f_l <= f_k * (1 + 1e-3)).float().mean().item() >= 0.75


def test_config5_family_training_and_evaluation(hp):
    """The random-centre family the learned initializer is specified on (25
    fresh centres per sample in d = 32): scheduled multi-epoch training on
    method-made pairs lowers the held-out loss; on fresh cold samples every
    accepted proposal has a sample objective no larger than the K-means++
    seeding's, and every rejected one leaves exactly the K-means++ start
    and its Lloyd run.  The measured acceptance, passes and final objective
    are printed (the gain is measured, not assumed)."""
    from paper_2311_04517_amd import learned

    d, k, s, n_enc = 32, 25, 4000, 1024
    train, held = learned.Pairs(d, k, n_enc), learned.Pairs(d, k, n_enc)
    for q, n_q, dst in ((0, 1024, train), (1, 1024, train), (2, 256, held)):
        X, idx, desc, idx_len, c_len = _family(hp, n_q, s, d, k, seed=500 + q)
        T, _, _ = learned.method_targets(X, idx, desc, c_len)
        dst.add(X, idx, desc, T)
        del X, idx, T
    train.finish()
    held.finish()
    assert (train.n, held.n) == (2048, 256)
    model = hp.SetEncoder(d, k, n_enc=n_enc, max_batch=64, seed=1)
    curve = learned.fit(model, train, held, epochs=4, batch=64, lr=2e-3, lr_min=2e-5, warmup=20)
    losses = [c["heldout"] for c in curve]
    assert np.isfinite(losses).all() and losses[-1] < losses[0], losses
    X, idx, desc, idx_len, c_len = _family(hp, 256, s, d, k, seed=777)
    ev = learned.evaluate(model, X, idx, desc, c_len)
    acc = ev["accepted"].astype(bool)
    assert np.array_equal(acc, ev["f_prop"] <= ev["f_kpp"])
    assert np.array_equal(ev["learned"]["passes"][~acc], ev["kmeanspp"]["passes"][~acc])
    assert np.array_equal(ev["learned"]["f"][~acc], ev["kmeanspp"]["f"][~acc])
    for name in ("learned", "kmeanspp", "proposal"):
        assert (ev[name]["passes"] >= 1).all() and np.isfinite(ev[name]["f"]).all()
    summ = learned.summarize(ev)
    print(f"config-5 family: held-out loss {losses}; evaluation {summ}")
