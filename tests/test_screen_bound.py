"""The screening error bound of every precision mode, checked on the CPU.

The kernels accept a screened nearest centroid only when its lead exceeds
a multiple of E(x) = alpha |x| cmax + beta cmax^2 (hpc_screen_bound), so
E must bound the difference between the screened score and the exact
score |c|^2 - 2 x.c.  Here the matrix cores' arithmetic is emulated
(operands rounded or split to BF16 as the kernels do, products exact for
BF16 operands and rounded or fused for FP32, FP32 accumulation from the
rounded |c|^2 in several summation orders) on random data and on
adversarial data where every rounding error has the same sign, and the
worst error is compared with E.  The adversarial cases also show the BF16
and BF16x3 bounds are not vacuous: with a quarter of alpha they fail.
"""
import numpy as np
import pytest
import torch

from paper_2311_04517_amd import _lib, api

PRECS = [(api.PREC_FP32, "fp32"), (api.PREC_BF16_MFMA, "bf16"), (api.PREC_BF16X3_MFMA, "bf16x3")]


@pytest.fixture(scope="module", autouse=True)
def _built():
    import os

    if not os.path.exists(_lib.LIB_PATH):
        from paper_2311_04517_amd import build

        build.build()


def bf16(a):
    """Round to nearest even BF16, returned as float32."""
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32))
    return t.to(torch.bfloat16).to(torch.float32).numpy()


def products(X, C, prec, fused=False):
    """float32 (n, k, T) terms the matrix cores add for -2 x.c, and |c|^2
    rounded to FP32."""
    a = (np.float32(-2.0) * C.astype(np.float32)).astype(np.float32)  # -2 fl32(c)
    nrm = (C * C).sum(1).astype(np.float32)
    if prec == api.PREC_FP32:
        if fused:  # exact products, rounded when added
            P = X.astype(np.float64)[:, None, :] * a.astype(np.float64)[None, :, :]
        else:
            P = (X[:, None, :] * a[None, :, :]).astype(np.float32)
    elif prec == api.PREC_BF16_MFMA:
        P = bf16(X)[:, None, :] * bf16(a)[None, :, :]  # exact in float32
    else:
        xh, ah = bf16(X), bf16(a)
        xl, al = bf16(X - xh), bf16(a - ah)  # the differences are exact in float32
        P = np.concatenate([al[None] * xh[:, None], ah[None] * xl[:, None],
                            ah[None] * xh[:, None]], axis=2)
    return P, nrm


def accumulate(P, nrm, order):
    """FP32 sum of nrm and the terms along the last axis."""
    n, k, T = P.shape
    start = np.broadcast_to(nrm, (n, k)).astype(np.float32)
    if order in ("seq", "rev"):
        acc = start.copy()
        for t in (range(T) if order == "seq" else range(T - 1, -1, -1)):
            acc = (acc.astype(np.float64) + P[:, :, t]).astype(np.float32)
        return acc
    if order == "tree":
        S = P.astype(np.float32)
        while S.shape[2] > 1:
            if S.shape[2] % 2:
                S = np.concatenate([S, np.zeros((n, k, 1), np.float32)], axis=2)
            S = (S[:, :, 0::2] + S[:, :, 1::2]).astype(np.float32)
        return (start + S[:, :, 0]).astype(np.float32)
    # chunks of 8 summed first, then added one after another
    acc = start.copy()
    for c0 in range(0, T, 8):
        part = np.zeros((n, k), np.float32)
        for t in range(c0, min(T, c0 + 8)):
            part = (part.astype(np.float64) + P[:, :, t]).astype(np.float32)
        acc = (acc + part).astype(np.float32)
    return acc


def worst_ratio(X, C, prec, alpha_scale=1.0):
    d = X.shape[1]
    alpha, beta = api.screen_bound(d, prec)
    Xl, Cl = X.astype(np.longdouble), C.astype(np.longdouble)
    exact = (Cl * Cl).sum(1)[None, :] - 2 * (Xl @ Cl.T)
    cmax = float(np.sqrt((C * C).sum(1).max()))
    E = (alpha_scale * alpha * np.sqrt((X.astype(np.float64) ** 2).sum(1)) * cmax
         + beta * cmax * cmax)[:, None]
    worst = 0.0
    for fused in ((False, True) if prec == api.PREC_FP32 else (False,)):
        P, nrm = products(X, C, prec, fused)
        for order in ("seq", "rev", "tree", "chunk8"):
            err = np.abs(accumulate(P, nrm, order).astype(np.longdouble) - exact)
            worst = max(worst, float((err / E).max()))
    return worst


def _random_case(d, seed):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-20, 20, size=(8, d))
    X = (centres[rng.integers(0, 8, 256)] + rng.normal(0, 2.0, (256, d))).astype(np.float32)
    C = X[rng.integers(0, 256, 24)].astype(np.float64) + rng.normal(0, 0.3, (24, d))
    return X, C


def _adversarial_case(d, seed):
    """Coordinates just below a BF16 rounding midpoint (rounded down by the
    largest relative amount), x and c of equal signs, magnitudes spread over
    a few binades: every operand error shrinks every product."""
    rng = np.random.default_rng(seed)
    sign = rng.choice([-1.0, 1.0], size=d)
    mant = 1.0 + 2.0 ** -8 - 2.0 ** -21
    X = (sign * mant * 2.0 ** rng.integers(0, 3, size=(64, d))).astype(np.float32)
    C = sign * mant * 2.0 ** rng.integers(0, 3, size=(16, d)) / 2.0
    return X, C


def _adversarial_split_case(d, seed):
    """The same for the BF16x3 split: the high part rounds to 1 and the
    remainder (just under 2^-8) sits just below a BF16 midpoint, so the low
    part drops the largest share of it, and the omitted lo.lo product has
    the sign of the products: all three error terms shrink every product."""
    rng = np.random.default_rng(seed)
    sign = rng.choice([-1.0, 1.0], size=d)
    mant = 1.0 + 2.0 ** -8 - 2.0 ** -17 - 2.0 ** -22
    X = (sign * mant * 2.0 ** rng.integers(0, 3, size=(64, d))).astype(np.float32)
    C = sign * mant * 2.0 ** rng.integers(0, 3, size=(16, d)) / 2.0
    return X, C


@pytest.mark.parametrize("prec,name", PRECS)
@pytest.mark.parametrize("d", [3, 16, 32, 64, 100, 128])
def test_screening_error_within_bound(prec, name, d):
    for case in (_random_case(d, d), _adversarial_case(d, d), _adversarial_split_case(d, d)):
        r = worst_ratio(*case, prec)
        assert r <= 1.0, f"{name} d={d}: screening error {r:.3f} x the bound"


@pytest.mark.parametrize("prec,name,case", [(api.PREC_BF16_MFMA, "bf16", _adversarial_case),
                                            (api.PREC_BF16X3_MFMA, "bf16x3",
                                             _adversarial_split_case)])
def test_bf16_bounds_are_not_vacuous(prec, name, case):
    """At d = 16, where the operand-rounding term dominates the bound, the
    adversarial errors exceed the bound with a quarter of alpha."""
    X, C = case(16, 5)
    assert worst_ratio(X, C, prec, alpha_scale=0.25) > 1.0, name


def test_bound_coefficients_order():
    """BF16x3's bound sits between FP32's and BF16's (d = 64)."""
    a32, b32 = api.screen_bound(64, api.PREC_FP32)
    a16, b16 = api.screen_bound(64, api.PREC_BF16_MFMA)
    a3, b3 = api.screen_bound(64, api.PREC_BF16X3_MFMA)
    assert a32 < a3 < a16 and a3 < a16 / 50
    with pytest.raises(_lib.HpcError):
        api.screen_bound(0, api.PREC_FP32)
    with pytest.raises(_lib.HpcError):
        api.screen_bound(8, 3)
