"""Parity tolerances between the gfx950 path and the FP64 oracle.

The GPU path stores data and returned centroids in FP32 but takes every
decision the method makes -- nearest centroid, K-means++ draw, best
candidate, stop test -- on FP64 values: FP32 screening with a rigorous
error certificate, FP64 re-decision of uncertified points, FP64 D^2,
potentials, sums, objectives and in-kernel centroids.  GPU and oracle FP64
values then differ only by summation order (~1e-16 relative per term); the
GPU's pass objective, taken from the running sums, is within ~1e-12
relative of the direct sum (it falls back to the direct sum where the
identity would cancel).

CLEAN_MARGIN   a decision whose oracle margin is below this may differ from
               the GPU's by summation-order noise; a run is "clean" when no
               decision is that close (1e-10, far above s * 1e-16).
TIE_REL        relative top-2 gap (d2 - d1)/d2 within which a label may
               differ (the build target states 1e-5; the GPU meets far less).
F_REL, SSE_REL relative tolerance on sample objectives and full SSE (1e-6).
C_REL          centroid rows: |c_gpu - c_orc| <= C_REL * (|c_orc| + sigma_S),
               sigma_S the RMS spread of the sample (1e-5); the GPU's
               centroids are FP64 values rounded to FP32 (6e-8).
"""
import numpy as np

CLEAN_MARGIN = 1e-10
TIE_REL = 1e-5
F_REL = 1e-6
SSE_REL = 1e-6
C_REL = 1e-5


def diag_clean(g: dict) -> bool:
    """No decision of the run sat within rounding of its threshold."""
    return (g["min_label_margin"] >= CLEAN_MARGIN and g["min_draw_margin"] >= CLEAN_MARGIN
            and g["min_cand_margin"] >= CLEAN_MARGIN and g["min_stop_margin"] >= CLEAN_MARGIN)


def assert_labels(gpu, orc, margins, what="labels"):
    """Bit-exact labels except points whose oracle top-2 relative gap is
    below TIE_REL.  Returns the number of exempt points."""
    gpu = np.asarray(gpu)
    orc = np.asarray(orc)
    margins = np.asarray(margins)
    diff = gpu != orc
    exempt = margins < TIE_REL
    bad = np.flatnonzero(diff & ~exempt)
    assert bad.size == 0, f"{what}: {bad.size} non-tie mismatches, e.g. index {bad[:5]}"
    return int(exempt.sum())


def assert_centroids(Cg, Co, S, what="centroids"):
    Cg = np.asarray(Cg, dtype=np.float64)
    Co = np.asarray(Co, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    sigma = np.sqrt(((S - S.mean(axis=0)) ** 2).sum(axis=1).mean())
    err = np.linalg.norm(Cg - Co, axis=1)
    lim = C_REL * (np.linalg.norm(Co, axis=1) + sigma)
    assert np.isfinite(Cg).all(), f"{what}: non-finite rows"
    assert (err <= lim).all(), f"{what}: max err/limit {np.max(err / lim):.3g}"


def rel(a, b):
    return abs(float(a) - float(b)) / max(abs(float(b)), 1e-300)
