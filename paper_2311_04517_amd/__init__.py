"""MI355X (gfx950) hot path of the sample-based MSSC method HPClust
(arXiv 2311.04517): sample draw, K-means++ seeding, Lloyd passes with
degenerate re-seeding, keep-the-best, and the full-data assignment with its
FP64 objective, as hand-written HIP kernels behind a C ABI
(include/hpclust.h).  This package is the thin Python binding."""
from .api import *  # noqa: F401,F403
from .api import __all__ as _api_all

__all__ = list(_api_all)
