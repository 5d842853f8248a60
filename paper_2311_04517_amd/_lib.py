"""ctypes loader for ``libhpclust.so`` (the gfx950 HIP library).

There is no fallback: if the library has not been built, or cannot be
loaded, every call raises.  Build it with ``python -m
paper_2311_04517_amd.build`` or ``__graft_entry__.build()``.
"""
from __future__ import annotations

import ctypes as ct
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhpclust.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hpclust.h")

HPC_OK = 0
HPC_ERR_INVALID_ARG = -1
HPC_ERR_HIP = -2
HPC_ERR_NO_MEMORY = -3
HPC_ERR_UNSUPPORTED = -4
PREC_FP32 = 0
PREC_BF16_MFMA = 1
PREC_BF16X3_MFMA = 2


class SampleDesc(ct.Structure):
    """Mirror of ``hpc_sample_desc``."""

    _fields_ = [
        ("idx_offset", ct.c_int64),
        ("c_offset", ct.c_int64),
        ("s", ct.c_int32),
        ("k", ct.c_int32),
        ("seed", ct.c_uint64),
        ("sample_id", ct.c_uint64),
    ]


class Tune(ct.Structure):
    """Mirror of ``hpc_tune``."""

    _fields_ = [
        ("wg_per_cu", ct.c_int32),
        ("copies", ct.c_int32),
        ("order", ct.c_int32),
        ("seed_team", ct.c_int32),
        ("seed_inflight", ct.c_int32),
        ("parts", ct.c_int32),
    ]

    def as_dict(self):
        return {"wg_per_cu": self.wg_per_cu, "copies": self.copies, "order": self.order,
                "seed_team": self.seed_team, "seed_inflight": self.seed_inflight,
                "parts": self.parts}


class HpcError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: status {code}: {msg}")
        self.code = code


_lib = None

_p = ct.c_void_p
_i32, _i64, _u32, _u64, _f64 = ct.c_int32, ct.c_int64, ct.c_uint32, ct.c_uint64, ct.c_double
_SIGS = {
    "hpc_version": ([], ct.c_char_p),
    "hpc_last_error": ([], ct.c_char_p),
    "hpc_device_count": ([], ct.c_int),
    "hpc_release": ([], ct.c_int),
    "hpc_draw_sample": ([_i64, _i32, _u64, _u64, _p, _p], ct.c_int),
    "hpc_draw_samples": ([_i64, _p, _i32, _p, _i64, _p], ct.c_int),
    "hpc_seed_kmeanspp": ([_p, _i64, _i32, _p, _i32, _i32, _i32, _u64, _u64, _u32, _p, _p, _p],
                          ct.c_int),
    "hpc_lloyd_batch": ([_p, _i64, _i32, _p, _i64, _p, _i32, _p, _i64, _i32, _f64, _i32, _p, _p,
                         _p, _p], ct.c_int),
    "hpc_keep_best": ([_p, _p, _p, _p, _i32, _i32, _i32, _p, _p], ct.c_int),
    "hpc_select_best": ([_p, _p, _i32, _i32, _i32, _p, _p, _p, _p], ct.c_int),
    "hpc_assign_sse": ([_p, _i64, _i32, _p, _i32, _i32, _p, _p, _p, _p], ct.c_int),
    "hpc_assign_sse_noalloc": ([_p, _i64, _i32, _p, _i32, _i32, _p, _p, _p, _p], ct.c_int),
    "hpc_screen_bound": ([_i32, _i32, _p, _p], ct.c_int),
    "hpc_plan_create": ([_i32, _p, _i32, _i64, _i64, _i32, ct.POINTER(_p)], ct.c_int),
    "hpc_plan_destroy": ([_p], ct.c_int),
    "hpc_plan_set_tune": ([_p, _p], ct.c_int),
    "hpc_plan_get_tune": ([_p, _p], ct.c_int),
    "hpc_plan_tune_key": ([_p, ct.c_char_p, _i32], ct.c_int),
    "hpc_plan_autotune": ([_p, _p, _i64, _p, _p, _i32, _f64, _p, _p, _p], ct.c_int),
    "hpc_plan_lloyd": ([_p, _p, _i64, _p, _p, _i32, _f64, _p, _p, _p, _p], ct.c_int),
    "hpc_plan_draw": ([_p, _i64, _p, _p], ct.c_int),
    "hpc_plan_advance": ([_p, _u64, _p], ct.c_int),
    "hpc_plan_round": ([_p, _p, _i64, _p, _p, _p, _p, _i32, _f64, _p, _p, _u64, _p], ct.c_int),
    "hpc_plan_capture_round": ([_p, _p, _i64, _p, _p, _p, _p, _i32, _f64, _p, _p, _u64],
                               ct.c_int),
    "hpc_plan_replay": ([_p, _i32, _p], ct.c_int),
    "hpc_plan_reset_ids": ([_p, _p], ct.c_int),
    "hpc_setenc_create": ([_i32, _i32, _i32, _i32, _u64, ct.POINTER(_p)], ct.c_int),
    "hpc_setenc_destroy": ([_p], ct.c_int),
    "hpc_setenc_param_count": ([_p, ct.POINTER(_i64)], ct.c_int),
    "hpc_setenc_get_params": ([_p, _i32, _p], ct.c_int),
    "hpc_setenc_set_params": ([_p, _p], ct.c_int),
    "hpc_setenc_get_grads": ([_p, _p], ct.c_int),
    "hpc_setenc_propose": ([_p, _p, _i64, _p, _i64, _p, _i32, _p, _i64, _p], ct.c_int),
    "hpc_setenc_grad": ([_p, _p, _i64, _p, _i64, _p, _i32, _p, _i64, _p, _p], ct.c_int),
    "hpc_setenc_adam": ([_p, ct.c_float, _p], ct.c_int),
    "hpc_learned_seed": ([_p, _p, _i64, _p, _i64, _p, _i32, _p, _p, _i64, _i32, _p, _p, _p, _p],
                         ct.c_int),
}


def header_functions() -> list[str]:
    """Names of the functions declared in include/hpclust.h."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hpc_[a-z_0-9]+)\s*\(", src)))


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: the HIP library has not been built "
            "(run `python -m paper_2311_04517_amd.build`)")
    L = ct.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def check(code: int, where: str):
    if code != HPC_OK:
        msg = lib().hpc_last_error().decode(errors="replace")
        raise HpcError(code, where, msg)
