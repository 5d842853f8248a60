"""Python binding of the C ABI (include/hpclust.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the method runs in the library's gfx950
kernels.  Function names follow the C entry points without the ``hpc_``
prefix.
"""
from __future__ import annotations

import ctypes as ct

import numpy as np
import torch

from ._lib import PREC_BF16_MFMA, PREC_FP32, SampleDesc, check, lib

__all__ = [
    "PREC_FP32", "PREC_BF16_MFMA", "SampleDesc", "make_desc", "draw_sample", "draw_samples",
    "seed_kmeanspp", "lloyd_batch", "keep_best", "select_best", "assign_sse", "release",
    "version",
]


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def version() -> str:
    return lib().hpc_version().decode()


def release():
    check(lib().hpc_release(), "hpc_release")


def make_desc(s, k, *, seed, sample_id, d: int, idx_offset=None, c_offset=None):
    """Descriptor table (host, ctypes array) for samples packed back to back.

    ``s``, ``k``, ``seed`` and ``sample_id`` are per-sample sequences (a
    scalar ``seed`` applies to all).  Returns (desc, idx_len, c_len)."""
    s = np.asarray(s, dtype=np.int64).ravel()
    k = np.asarray(k, dtype=np.int64).ravel()
    n = len(s)
    if k.size == 1 and n > 1:
        k = np.full(n, int(k[0]))
    seed = np.broadcast_to(np.asarray(seed, dtype=np.uint64), (n,))
    sample_id = np.asarray(sample_id, dtype=np.uint64).ravel()
    io = np.concatenate([[0], np.cumsum(s)[:-1]]) if idx_offset is None else np.asarray(idx_offset)
    co = (np.concatenate([[0], np.cumsum(k * d)[:-1]]) if c_offset is None
          else np.asarray(c_offset))
    desc = (SampleDesc * n)()
    for b in range(n):
        desc[b].idx_offset = int(io[b])
        desc[b].c_offset = int(co[b])
        desc[b].s = int(s[b])
        desc[b].k = int(k[b])
        desc[b].seed = int(seed[b])
        desc[b].sample_id = int(sample_id[b])
    idx_len = int(max(io[b] + s[b] for b in range(n)))
    c_len = int(max(co[b] + k[b] * d for b in range(n)))
    return desc, idx_len, c_len


def draw_sample(m: int, s: int, seed: int, sample_id: int, *, out=None, device="cuda"):
    idx = out if out is not None else torch.empty(s, dtype=torch.int64, device=device)
    _dev(idx, torch.int64, "idx")
    check(lib().hpc_draw_sample(m, s, seed, sample_id, _ptr(idx), ct.c_void_p(_stream())),
          "hpc_draw_sample")
    return idx


def draw_samples(m: int, desc, idx_len: int, *, out=None, device="cuda"):
    idx = out if out is not None else torch.empty(idx_len, dtype=torch.int64, device=device)
    _dev(idx, torch.int64, "idx")
    check(lib().hpc_draw_samples(m, desc, len(desc), _ptr(idx), idx.numel(),
                                 ct.c_void_p(_stream())), "hpc_draw_samples")
    return idx


def seed_kmeanspp(X, idx, k: int, *, seed: int, sample_id: int = 0, call_id: int = 0,
                  n_cand: int = 3, C=None, want_chosen=True):
    _dev(X, torch.float32, "X")
    _dev(idx, torch.int64, "idx")
    m, d = X.shape
    if C is None:
        C = torch.full((k, d), float("nan"), dtype=torch.float32, device=X.device)
    _dev(C, torch.float32, "C")
    chosen = torch.empty(k, dtype=torch.int32, device=X.device) if want_chosen else None
    check(lib().hpc_seed_kmeanspp(_ptr(X), m, d, _ptr(idx), idx.numel(), k, n_cand, seed,
                                  sample_id, call_id, _ptr(C), _ptr(chosen),
                                  ct.c_void_p(_stream())), "hpc_seed_kmeanspp")
    return C, chosen


def lloyd_batch(X, idx, desc, C, *, max_iter=300, rel_tol=1e-4, precision=PREC_FP32,
                want_labels=False, f_out=None, iters_out=None, labels_out=None):
    """K-means on every sample of ``desc`` (in place on ``C``).
    Returns (f, iters, labels)."""
    _dev(X, torch.float32, "X")
    _dev(idx, torch.int64, "idx")
    _dev(C, torch.float32, "C")
    m, d = X.shape
    n = len(desc)
    f = f_out if f_out is not None else torch.empty(n, dtype=torch.float64, device=X.device)
    it = iters_out if iters_out is not None else torch.empty(n, dtype=torch.int32, device=X.device)
    lab = labels_out
    if want_labels and lab is None:
        lab = torch.empty(idx.numel(), dtype=torch.int32, device=X.device)
    check(lib().hpc_lloyd_batch(_ptr(X), m, d, _ptr(idx), idx.numel(), desc, n, _ptr(C),
                                C.numel(), max_iter, rel_tol, precision, _ptr(f), _ptr(it),
                                _ptr(lab), ct.c_void_p(_stream())), "hpc_lloyd_batch")
    return f, it, lab


def keep_best(C_new, f_new, C_inc, f_inc, k: int, d: int, *, want_updated=False):
    n = f_inc.numel()
    upd = torch.empty(n, dtype=torch.int32, device=f_inc.device) if want_updated else None
    check(lib().hpc_keep_best(_ptr(C_new), _ptr(f_new), _ptr(C_inc), _ptr(f_inc), n, k, d,
                              _ptr(upd), ct.c_void_p(_stream())), "hpc_keep_best")
    return upd


def select_best(C_inc, f_inc, k: int, d: int):
    n = f_inc.numel()
    Cb = torch.empty((k, d), dtype=torch.float32, device=f_inc.device)
    fb = torch.empty(1, dtype=torch.float64, device=f_inc.device)
    wb = torch.empty(1, dtype=torch.int32, device=f_inc.device)
    check(lib().hpc_select_best(_ptr(C_inc), _ptr(f_inc), n, k, d, _ptr(Cb), _ptr(fb), _ptr(wb),
                                ct.c_void_p(_stream())), "hpc_select_best")
    return Cb, fb, wb


def assign_sse(X, C, *, want_labels=True, want_counts=True, precision=PREC_FP32, labels=None,
               counts=None, sse=None):
    _dev(X, torch.float32, "X")
    _dev(C, torch.float32, "C")
    m, d = X.shape
    k = C.shape[0]
    if want_labels and labels is None:
        labels = torch.empty(m, dtype=torch.int32, device=X.device)
    if want_counts and counts is None:
        counts = torch.empty(k, dtype=torch.int64, device=X.device)
    if sse is None:
        sse = torch.empty(1, dtype=torch.float64, device=X.device)
    check(lib().hpc_assign_sse(_ptr(X), m, d, _ptr(C), k, precision, _ptr(labels), _ptr(counts),
                               _ptr(sse), ct.c_void_p(_stream())), "hpc_assign_sse")
    return labels, counts, sse
