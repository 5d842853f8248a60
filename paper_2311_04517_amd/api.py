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

from ._lib import PREC_BF16_MFMA, PREC_BF16X3_MFMA, PREC_FP32, SampleDesc, Tune, check, lib

__all__ = [
    "PREC_FP32", "PREC_BF16_MFMA", "PREC_BF16X3_MFMA", "SampleDesc", "make_desc", "draw_sample",
    "draw_samples", "seed_kmeanspp", "lloyd_batch", "keep_best", "select_best", "assign_sse",
    "screen_bound", "release", "version", "Plan", "Tune", "SetEncoder",
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


def screen_bound(d: int, precision=PREC_FP32):
    """(alpha, beta) of the screening error bound the kernels use for
    dimension d: |s~ - s| <= alpha |x| cmax + beta cmax^2 (host only)."""
    a, b = ct.c_double(), ct.c_double()
    check(lib().hpc_screen_bound(d, precision, ct.byref(a), ct.byref(b)), "hpc_screen_bound")
    return a.value, b.value


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


class Plan:
    """A prepared batch of (possibly uneven) samples: ``hpc_plan_*``.

    Holds the library's plan handle; the device buffers it owns are freed by
    :meth:`close` (or on garbage collection)."""

    def __init__(self, d: int, desc, idx_len: int, c_len: int, precision=PREC_FP32):
        self.d, self.n, self.idx_len, self.c_len = d, len(desc), idx_len, c_len
        self.precision = precision
        self._desc = desc
        h = ct.c_void_p()
        check(lib().hpc_plan_create(d, desc, len(desc), idx_len, c_len, precision, ct.byref(h)),
              "hpc_plan_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            check(lib().hpc_plan_destroy(self._h), "hpc_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def tune(self) -> Tune:
        t = Tune()
        check(lib().hpc_plan_get_tune(self._h, ct.byref(t)), "hpc_plan_get_tune")
        return t

    def set_tune(self, wg_per_cu=0, copies=0, order=0, seed_team=0, seed_inflight=0, parts=0):
        t = Tune(wg_per_cu, copies, order, seed_team, seed_inflight, parts)
        check(lib().hpc_plan_set_tune(self._h, ct.byref(t)), "hpc_plan_set_tune")

    def tune_key(self) -> str:
        buf = ct.create_string_buffer(256)
        check(lib().hpc_plan_tune_key(self._h, buf, 256), "hpc_plan_tune_key")
        return buf.value.decode()

    def autotune(self, X, idx, C, *, max_iter=3, rel_tol=0.0):
        """Time every launch configuration on these inputs (Lloyd from C,
        max_iter passes, stop rule rel_tol; 0 = exactly max_iter) and keep
        the fastest (synchronous).  Returns (Tune, ms)."""
        _dev(X, torch.float32, "X")
        _dev(idx, torch.int64, "idx")
        _dev(C, torch.float32, "C")
        t = Tune()
        ms = ct.c_double()
        check(lib().hpc_plan_autotune(self._h, _ptr(X), X.shape[0], _ptr(idx), _ptr(C), max_iter,
                                      rel_tol, ct.byref(t), ct.byref(ms), ct.c_void_p(_stream())),
              "hpc_plan_autotune")
        return t, ms.value

    def lloyd(self, X, idx, C, *, max_iter=300, rel_tol=1e-4, want_labels=False, f_out=None,
              iters_out=None, labels_out=None):
        _dev(X, torch.float32, "X")
        _dev(idx, torch.int64, "idx")
        _dev(C, torch.float32, "C")
        self._lengths(idx, C)
        f = f_out if f_out is not None else torch.empty(self.n, dtype=torch.float64,
                                                         device=X.device)
        it = iters_out if iters_out is not None else torch.empty(self.n, dtype=torch.int32,
                                                                  device=X.device)
        lab = labels_out
        if want_labels and lab is None:
            lab = torch.empty(self.idx_len, dtype=torch.int32, device=X.device)
        check(lib().hpc_plan_lloyd(self._h, _ptr(X), X.shape[0], _ptr(idx), _ptr(C), max_iter,
                                   rel_tol, _ptr(f), _ptr(it), _ptr(lab), ct.c_void_p(_stream())),
              "hpc_plan_lloyd")
        return f, it, lab

    def draw(self, m: int, idx):
        """Draw every sample with the plan's current sample ids."""
        _dev(idx, torch.int64, "idx")
        if idx.numel() < self.idx_len:
            raise ValueError("idx shorter than the plan's idx_len")
        check(lib().hpc_plan_draw(self._h, m, _ptr(idx), ct.c_void_p(_stream())), "hpc_plan_draw")
        return idx

    def advance(self, id_stride=None):
        """sample_id += id_stride (default n) in the plan's device table."""
        stride = self.n if id_stride is None else id_stride
        check(lib().hpc_plan_advance(self._h, stride, ct.c_void_p(_stream())), "hpc_plan_advance")

    def _lengths(self, idx, C, C_inc=None, f_inc=None):
        if idx.numel() < self.idx_len or C.numel() < self.c_len:
            raise ValueError("idx / C shorter than the plan's idx_len / c_len")
        if C_inc is not None and C_inc.numel() < self.c_len:
            raise ValueError("C_inc shorter than the plan's c_len")
        if f_inc is not None and f_inc.numel() < self.n:
            raise ValueError("f_inc shorter than the number of samples")

    def _round_args(self, X, idx, C, C_inc, f_inc, f_out, iters_out):
        for t, dt, name in ((X, torch.float32, "X"), (idx, torch.int64, "idx"),
                            (C, torch.float32, "C"), (C_inc, torch.float32, "C_inc"),
                            (f_inc, torch.float64, "f_inc"), (f_out, torch.float64, "f_out"),
                            (iters_out, torch.int32, "iters_out")):
            _dev(t, dt, name)
        self._lengths(idx, C, C_inc, f_inc)
        if f_out.numel() < self.n or iters_out.numel() < self.n:
            raise ValueError("f_out / iters_out shorter than the number of samples")
        return (_ptr(X), X.shape[0], _ptr(idx), _ptr(C), _ptr(C_inc), _ptr(f_inc))

    def round(self, X, idx, C, C_inc, f_inc, f_out, iters_out, *, max_iter=300, rel_tol=1e-4,
              id_stride=None):
        """One worker-loop round (draw, start from incumbents, Lloyd, keep
        the best, advance sample ids by ``id_stride``, default n)."""
        a = self._round_args(X, idx, C, C_inc, f_inc, f_out, iters_out)
        stride = self.n if id_stride is None else id_stride
        check(lib().hpc_plan_round(self._h, *a, max_iter, rel_tol, _ptr(f_out), _ptr(iters_out),
                                   stride, ct.c_void_p(_stream())), "hpc_plan_round")

    def capture_round(self, X, idx, C, C_inc, f_inc, f_out, iters_out, *, max_iter=300,
                      rel_tol=1e-4, id_stride=None):
        a = self._round_args(X, idx, C, C_inc, f_inc, f_out, iters_out)
        stride = self.n if id_stride is None else id_stride
        self._keep = (X, idx, C, C_inc, f_inc, f_out, iters_out)  # buffers the graph uses
        check(lib().hpc_plan_capture_round(self._h, *a, max_iter, rel_tol, _ptr(f_out),
                                           _ptr(iters_out), stride), "hpc_plan_capture_round")

    def replay(self, n_rounds=1):
        check(lib().hpc_plan_replay(self._h, n_rounds, ct.c_void_p(_stream())), "hpc_plan_replay")

    def reset_ids(self):
        check(lib().hpc_plan_reset_ids(self._h, ct.c_void_p(_stream())), "hpc_plan_reset_ids")


class SetEncoder:
    """The learned initializer's model (``hpc_setenc_*``): a set encoder
    proposing k x d starting centroids per sample."""

    PARAM_NAMES = ("W1", "b1", "W2", "b2", "Wh", "bh")
    H = 256

    def __init__(self, d: int, k: int, *, n_enc: int = 1024, max_batch: int = 64, seed: int = 0):
        self.d, self.k, self.n_enc, self.max_batch = d, k, n_enc, max_batch
        h = ct.c_void_p()
        check(lib().hpc_setenc_create(d, k, n_enc, max_batch, seed, ct.byref(h)),
              "hpc_setenc_create")
        self._h = h
        n = ct.c_int64()
        check(lib().hpc_setenc_param_count(h, ct.byref(n)), "hpc_setenc_param_count")
        self.n_params = n.value

    def close(self):
        if getattr(self, "_h", None):
            check(lib().hpc_setenc_destroy(self._h), "hpc_setenc_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def shapes(self) -> dict:
        H, d, kd = self.H, self.d, self.k * self.d
        return {"W1": (d, H), "b1": (H,), "W2": (H, H), "b2": (H,), "Wh": (H, kd), "bh": (kd,)}

    def _split(self, flat):
        out, off = {}, 0
        for name, shp in self.shapes().items():
            n = int(np.prod(shp))
            out[name] = flat[off:off + n].reshape(shp)
            off += n
        return out

    def get_params(self, rounded=False) -> dict:
        """Parameters as float32 numpy arrays (``rounded``: the BF16 values
        the kernels use for the weights)."""
        flat = np.empty(self.n_params, dtype=np.float32)
        check(lib().hpc_setenc_get_params(self._h, int(bool(rounded)),
                                          flat.ctypes.data_as(ct.c_void_p)),
              "hpc_setenc_get_params")
        return self._split(flat)

    def set_params(self, params: dict):
        flat = np.concatenate([np.asarray(params[n], dtype=np.float32).ravel()
                               for n in self.PARAM_NAMES])
        assert flat.size == self.n_params
        check(lib().hpc_setenc_set_params(self._h, flat.ctypes.data_as(ct.c_void_p)),
              "hpc_setenc_set_params")

    def get_grads(self) -> dict:
        flat = np.empty(self.n_params, dtype=np.float32)
        check(lib().hpc_setenc_get_grads(self._h, flat.ctypes.data_as(ct.c_void_p)),
              "hpc_setenc_get_grads")
        return self._split(flat)

    def propose(self, X, idx, desc, C):
        _dev(X, torch.float32, "X")
        _dev(idx, torch.int64, "idx")
        _dev(C, torch.float32, "C")
        check(lib().hpc_setenc_propose(self._h, _ptr(X), X.shape[0], _ptr(idx), idx.numel(), desc,
                                       len(desc), _ptr(C), C.numel(), ct.c_void_p(_stream())),
              "hpc_setenc_propose")
        return C

    def grad(self, X, idx, desc, T, loss=None):
        _dev(X, torch.float32, "X")
        _dev(idx, torch.int64, "idx")
        _dev(T, torch.float32, "T")
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device=X.device)
        check(lib().hpc_setenc_grad(self._h, _ptr(X), X.shape[0], _ptr(idx), idx.numel(), desc,
                                    len(desc), _ptr(T), T.numel(), _ptr(loss),
                                    ct.c_void_p(_stream())), "hpc_setenc_grad")
        return loss

    def adam(self, lr: float):
        check(lib().hpc_setenc_adam(self._h, ct.c_float(lr), ct.c_void_p(_stream())),
              "hpc_setenc_adam")

    def learned_seed(self, X, idx, desc, C, *, precision=PREC_FP32, C_kpp=None):
        """Seeds for a cold batch: the proposal where its sample objective
        is no larger than the K-means++ seeding's, else the seeding.
        Returns (C, C_kpp, f_prop, f_kpp, accepted)."""
        _dev(X, torch.float32, "X")
        _dev(idx, torch.int64, "idx")
        _dev(C, torch.float32, "C")
        n = len(desc)
        if C_kpp is None:
            C_kpp = torch.empty_like(C)
        fp = torch.empty(n, dtype=torch.float64, device=X.device)
        fk = torch.empty(n, dtype=torch.float64, device=X.device)
        acc = torch.empty(n, dtype=torch.int32, device=X.device)
        check(lib().hpc_learned_seed(self._h, _ptr(X), X.shape[0], _ptr(idx), idx.numel(), desc, n,
                                     _ptr(C), _ptr(C_kpp), C.numel(), precision, _ptr(fp),
                                     _ptr(fk), _ptr(acc), ct.c_void_p(_stream())),
              "hpc_learned_seed")
        return C, C_kpp, fp, fk, acc
