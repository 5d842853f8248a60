"""Cache of autotuned launch configurations for batch plans.

``hpc_plan_autotune`` times every configuration of the resident Lloyd
kernel on the caller's inputs; this module keeps the winners in a JSON file
keyed by ``hpc_plan_tune_key`` (device architecture, padded d, precision,
power-of-two buckets of batch size, largest k and mean s), so a plan of the
same shape reuses the result without timing again.
"""
from __future__ import annotations

import json
import os
import tempfile

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "hpclust", "tune.json")


def cache_path(path: str | None = None) -> str:
    return path or os.environ.get("HPCLUST_TUNE_CACHE") or DEFAULT_CACHE


def load(path: str | None = None) -> dict:
    p = cache_path(path)
    try:
        with open(p) as fh:
            db = json.load(fh)
        return db if isinstance(db, dict) else {}
    except (OSError, ValueError):
        return {}


def store(db: dict, path: str | None = None) -> None:
    p = cache_path(path)
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(p) or ".", suffix=".tmp")
    with os.fdopen(fd, "w") as fh:
        json.dump(db, fh, indent=1, sort_keys=True)
    os.replace(tmp, p)


def tuned(plan, X, idx, C, *, path: str | None = None, max_iter: int = 3, rel_tol: float = 0.0,
          retune: bool = False):
    """Give ``plan`` its cached configuration, or autotune it on (X, idx, C)
    (Lloyd from C with max_iter and rel_tol) and cache the result.  Returns
    (config dict, measured ms or None)."""
    key = plan.tune_key()
    db = load(path)
    ent = db.get(key)
    if ent is not None and not retune:
        cfg = {k: int(ent.get(k, 0)) for k in ("wg_per_cu", "copies", "order", "seed_team", "seed_inflight",
                                             "parts")}
        plan.set_tune(**cfg)
        return cfg, None
    t, ms = plan.autotune(X, idx, C, max_iter=max_iter, rel_tol=rel_tol)
    cfg = t.as_dict()
    db[key] = dict(cfg, ms=ms)
    try:
        store(db, path)
    except OSError as e:  # an unwritable cache costs a re-tune next time, nothing else
        import warnings

        warnings.warn(f"tuning cache not written: {e}")
    return cfg, ms
