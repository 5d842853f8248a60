"""FP64 CPU oracle for the sample-based MSSC method (HPClust, arXiv 2311.04517).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP path; the HIP path never imports it.

Thin ctypes wrappers around ``liboracle.so`` (built from ``hpc_oracle.c``);
every function takes and returns numpy arrays.  Centroids are k x d FP64,
row-major; a row whose first coordinate is NaN is degenerate.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

TAG_SAMPLE = 0
TAG_SEED = 1
TAG_RESEED = 2


class Diag(ct.Structure):
    _fields_ = [
        ("n_dist", ct.c_int64),
        ("n_seed_calls", ct.c_int64),
        ("n_seeded_rows", ct.c_int64),
        ("n_passes", ct.c_int64),
        ("n_zero_weight", ct.c_int64),
        ("n_label_ties", ct.c_int64),
        ("tie_rel", ct.c_double),
        ("min_label_margin", ct.c_double),
        ("min_draw_margin", ct.c_double),
        ("min_cand_margin", ct.c_double),
        ("min_stop_margin", ct.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def _new_diag(tie_rel: float) -> Diag:
    g = Diag()
    g.tie_rel = tie_rel
    lib().orc_diag_reset(ct.byref(g))
    return g


def lib():
    """Load ``liboracle.so``, building it first if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build_oracle

        build_oracle.build()
    L = ct.CDLL(_LIB_PATH)
    p = ct.c_void_p
    i32, i64, u64, f64 = ct.c_int32, ct.c_int64, ct.c_uint64, ct.c_double
    L.orc_philox4x64_10.argtypes = [p, p, p]
    L.orc_philox4x64_10.restype = None
    L.orc_diag_reset.argtypes = [p]
    L.orc_diag_reset.restype = None
    L.orc_draw_sample.argtypes = [i64, i32, u64, u64, p]
    L.orc_draw_sample.restype = None
    L.orc_kmeanspp.argtypes = [p, i64, i32, p, i32, i32, i32, u64, u64, u64, p, p, p]
    L.orc_kmeanspp.restype = ct.c_int
    L.orc_lloyd.argtypes = [p, i64, i32, p, i32, i32, i32, p, i32, f64, u64, u64, p, p, p, p, p]
    L.orc_lloyd.restype = ct.c_int
    L.orc_assign_sse.argtypes = [p, i64, i32, p, i32, p, p, p, p, p]
    L.orc_assign_sse.restype = ct.c_int
    L.orc_worker_loop.argtypes = [p, i64, i32, i32, i32, i32, i32, u64, i32, f64, p, p, p, p, p, p,
                                  p, p]
    L.orc_worker_loop.restype = ct.c_int
    L.orc_lloyd_batch.argtypes = [p, i64, i32, p, p, p, p, p, p, p, i32, i32, p, i32, f64, p, p, p,
                                  i32, p]
    L.orc_lloyd_batch.restype = ct.c_int
    L.orc_max_threads.argtypes = []
    L.orc_max_threads.restype = ct.c_int
    _lib = L
    return L


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _f32(X):
    X = np.ascontiguousarray(X, dtype=np.float32)
    assert X.ndim == 2
    return X


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def philox4x64_10(ctr, key) -> np.ndarray:
    """Four 64-bit words of Philox4x64-10 for counter ``ctr`` (4) and ``key`` (2)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def draw_sample(m: int, s: int, seed: int, sample_id: int) -> np.ndarray:
    """s i.i.d. uniform row indices in [0, m) for sample ``sample_id``."""
    idx = np.zeros(s, dtype=np.int64)
    lib().orc_draw_sample(m, s, seed, sample_id, _ptr(idx))
    return idx


def degenerate_centroids(k: int, d: int) -> np.ndarray:
    return np.full((k, d), np.nan, dtype=np.float64)


def kmeanspp(X, idx, k, *, seed, sample_id=0, call_id=0, n_cand=3, C=None, tie_rel=1e-5):
    """K-means++ (greedy, ``n_cand`` candidates) on the sample X[idx].

    Rows of ``C`` that are NaN are seeded; valid rows are kept and count as
    existing centres.  Returns (C, chosen, diag)."""
    X = _f32(X)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    d = X.shape[1]
    Cm = degenerate_centroids(k, d) if C is None else np.array(C, dtype=np.float64, order="C")
    chosen = np.zeros(k, dtype=np.int32)
    g = _new_diag(tie_rel)
    rc = lib().orc_kmeanspp(_ptr(X), X.shape[0], d, _ptr(idx), len(idx), k, n_cand, seed,
                            sample_id, call_id, _ptr(Cm), _ptr(chosen), ct.byref(g))
    _check(rc, "kmeanspp")
    return Cm, chosen, g.as_dict()


@dataclass
class LloydResult:
    C: np.ndarray
    f: float
    iters: int
    labels: np.ndarray
    margins: np.ndarray | None
    diag: dict


def lloyd(X, idx, k, C=None, *, seed, sample_id=0, max_iter=300, rel_tol=1e-4, n_cand=3,
          want_margins=False, tie_rel=1e-5) -> LloydResult:
    """K-means on the sample X[idx] from ``C`` (all-NaN = cold start)."""
    X = _f32(X)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    d = X.shape[1]
    Cm = degenerate_centroids(k, d) if C is None else np.array(C, dtype=np.float64, order="C")
    s = len(idx)
    labels = np.zeros(s, dtype=np.int32)
    margins = np.zeros(s, dtype=np.float64) if want_margins else None
    f = ct.c_double()
    it = ct.c_int32()
    g = _new_diag(tie_rel)
    rc = lib().orc_lloyd(_ptr(X), X.shape[0], d, _ptr(idx), s, k, n_cand, _ptr(Cm), max_iter,
                         rel_tol, seed, sample_id, _ptr(labels), ct.byref(f), ct.byref(it),
                         _ptr(margins), ct.byref(g))
    _check(rc, "lloyd")
    return LloydResult(Cm, f.value, it.value, labels, margins, g.as_dict())


def assign_sse(X, Cm, *, want_labels=True, want_margins=False, tie_rel=1e-5):
    """Nearest-centroid labels, per-cluster counts and the FP64 objective."""
    X = _f32(X)
    Cm = np.ascontiguousarray(Cm, dtype=np.float64)
    m, d = X.shape
    k = Cm.shape[0]
    labels = np.zeros(m, dtype=np.int32) if want_labels else None
    counts = np.zeros(k, dtype=np.int64)
    margins = np.zeros(m, dtype=np.float64) if want_margins else None
    sse = ct.c_double()
    g = _new_diag(tie_rel)
    rc = lib().orc_assign_sse(_ptr(X), m, d, _ptr(Cm), k, _ptr(labels), _ptr(counts),
                              ct.byref(sse), _ptr(margins), ct.byref(g))
    _check(rc, "assign_sse")
    return {"labels": labels, "counts": counts, "sse": sse.value, "margins": margins,
            "diag": g.as_dict()}


def worker_loop(X, *, s, k, n_samples, seed, max_iter=300, rel_tol=1e-4, n_cand=3,
                want_labels=True, tie_rel=1e-5):
    """One worker of Algorithm 3: keep-the-best over ``n_samples`` samples,
    then the final assignment of X."""
    X = _f32(X)
    m, d = X.shape
    C_w = np.zeros((k, d), dtype=np.float64)
    f_hat = ct.c_double()
    f_s = np.zeros(n_samples, dtype=np.float64)
    it_s = np.zeros(n_samples, dtype=np.int32)
    labels = np.zeros(m, dtype=np.int32) if want_labels else None
    counts = np.zeros(k, dtype=np.int64)
    sse = ct.c_double()
    g = _new_diag(tie_rel)
    rc = lib().orc_worker_loop(_ptr(X), m, d, s, k, n_cand, n_samples, seed, max_iter, rel_tol,
                               _ptr(C_w), ct.byref(f_hat), _ptr(f_s), _ptr(it_s), _ptr(labels),
                               _ptr(counts), ct.byref(sse), ct.byref(g))
    _check(rc, "worker_loop")
    return {"C": C_w, "f_hat": f_hat.value, "f_samples": f_s, "iters": it_s, "labels": labels,
            "counts": counts, "sse": sse.value, "diag": g.as_dict()}


def lloyd_batch(X, idx, desc, C, *, max_iter=300, rel_tol=1e-4, n_cand=3, want_labels=False,
                n_threads=1, tie_rel=1e-5):
    """Independent samples.  ``desc`` is a dict of arrays idx_offset, s, k,
    c_offset, seed, sample_id; ``C`` the concatenated FP64 centroid blocks
    (modified in place).  Returns f, iters, labels and per-sample diags."""
    X = _f32(X)
    m, d = X.shape
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    io = np.ascontiguousarray(desc["idx_offset"], dtype=np.int64)
    ss = np.ascontiguousarray(desc["s"], dtype=np.int32)
    kk = np.ascontiguousarray(desc["k"], dtype=np.int32)
    co = np.ascontiguousarray(desc["c_offset"], dtype=np.int64)
    sd = np.ascontiguousarray(desc["seed"], dtype=np.uint64)
    sid = np.ascontiguousarray(desc["sample_id"], dtype=np.uint64)
    n = len(ss)
    assert C.dtype == np.float64 and C.flags.c_contiguous
    f = np.zeros(n, dtype=np.float64)
    its = np.zeros(n, dtype=np.int32)
    labels = np.zeros(len(idx), dtype=np.int32) if want_labels else None
    diags = (Diag * n)()
    for b in range(n):
        diags[b].tie_rel = tie_rel
        lib().orc_diag_reset(ct.byref(diags[b]))
    rc = lib().orc_lloyd_batch(_ptr(X), m, d, _ptr(idx), _ptr(io), _ptr(ss), _ptr(kk), _ptr(co),
                               _ptr(sd), _ptr(sid), n, n_cand, _ptr(C), max_iter, rel_tol, _ptr(f),
                               _ptr(its), _ptr(labels), n_threads, diags)
    _check(rc, "lloyd_batch")
    return {"f": f, "iters": its, "labels": labels, "diag": [dg.as_dict() for dg in diags]}


def max_threads() -> int:
    return int(lib().orc_max_threads())
