"""Parity tolerances between the gfx950 path (FP32 distances, FP64 sums)
and the FP64 oracle.

TIE_REL        relative gap (d2 - d1)/d2 below which a point's assignment is
               exempt from bit-exact comparison (stated by the build's
               target: 1e-5).  An FP32 direct-difference distance over d
               coordinates has relative error at most about (d + 3) * 2^-24
               (4e-6 at d = 64), so outside the band the FP32 and FP64
               argmins agree.
DRAW_MARGIN    a K-means++ draw whose target lies closer than this fraction
               of the total weight to a prefix-sum boundary may pick the
               neighbouring index (FP32 D^2 vs FP64): same bound as above.
CAND_MARGIN    candidates whose potentials differ by less than this relative
               gap may be ranked differently.
STOP_MARGIN    a stop decision whose relative improvement lies within this
               absolute distance of rel_tol may fall the other way (the two
               objectives each carry the relative error above).
F_REL, SSE_REL relative tolerance on sample objectives and full SSE (1e-6).
C_REL          centroid rows: |c_gpu - c_orc| <= C_REL * (|c_orc| + sigma_S),
               sigma_S the RMS spread of the sample (1e-5).
"""
import numpy as np

TIE_REL = 1e-5
DRAW_MARGIN = 1e-5
CAND_MARGIN = 1e-5
STOP_MARGIN = 1e-5
F_REL = 1e-6
SSE_REL = 1e-6
C_REL = 1e-5


def diag_clean(g: dict) -> bool:
    """No decision of the run sat within rounding of its threshold."""
    return (g["min_label_margin"] >= TIE_REL and g["min_draw_margin"] >= DRAW_MARGIN
            and g["min_cand_margin"] >= CAND_MARGIN and g["min_stop_margin"] >= STOP_MARGIN)


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
