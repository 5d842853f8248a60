"""The C-ABI library loads, exports every declared entry point, and rejects
bad arguments on the host before anything touches a GPU (CPU-only)."""
import ctypes as ct
import os

import pytest

from paper_2311_04517_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2311_04517_amd import build

        build.build()
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = _lib.header_functions()
    assert {"hpc_seed_kmeanspp", "hpc_lloyd_batch", "hpc_assign_sse"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib._SIGS), "binding signatures must cover the header exactly"


def test_version(L):
    assert L.hpc_version().decode().startswith("hpclust-gfx950")


def _desc(*rows):
    d = (_lib.SampleDesc * len(rows))()
    for i, (io, co, s, k) in enumerate(rows):
        d[i].idx_offset, d[i].c_offset, d[i].s, d[i].k = io, co, s, k
        d[i].seed, d[i].sample_id = 1, i
    return d


P = ct.c_void_p(0x1000)  # never dereferenced: validation fails first


def _err(L, rc):
    assert rc == _lib.HPC_ERR_INVALID_ARG, rc
    assert L.hpc_last_error().decode()


def test_lloyd_batch_validation(L):
    good = _desc((0, 0, 10, 3))
    args = dict(X=P, m=100, d=4, idx=P, idx_len=10, desc=good, n=1, C=P, c_len=12, it=300,
                tol=1e-4, prec=0, f=P, its=P, lab=None, st=None)

    def call(**kw):
        a = dict(args, **kw)
        return L.hpc_lloyd_batch(a["X"], a["m"], a["d"], a["idx"], a["idx_len"], a["desc"], a["n"],
                                 a["C"], a["c_len"], a["it"], a["tol"], a["prec"], a["f"], a["its"],
                                 a["lab"], a["st"])

    _err(L, call(X=None))
    _err(L, call(f=None))
    _err(L, call(d=0))
    _err(L, call(d=129))
    _err(L, call(it=0))
    _err(L, call(tol=-1.0))
    _err(L, call(tol=float("nan")))
    _err(L, call(prec=7))
    _err(L, call(desc=_desc((0, 0, 2, 3))))              # s < k
    _err(L, call(desc=_desc((5, 0, 10, 3))))             # idx range beyond idx_len
    _err(L, call(desc=_desc((0, 4, 10, 3))))             # centroid block beyond c_len
    _err(L, call(desc=_desc((0, 0, 5, 3), (3, 12, 5, 3)), n=2, c_len=24))  # shared idx
    _err(L, call(desc=_desc((0, 0, 5, 3), (5, 6, 5, 3)), n=2, c_len=24))   # shared C


def test_seed_and_assign_and_draw_validation(L):
    _err(L, L.hpc_seed_kmeanspp(P, 100, 4, P, 10, 3, 5, 0, 0, 0, P, None, None))   # 5 candidates
    _err(L, L.hpc_seed_kmeanspp(P, 100, 4, P, 2, 3, 3, 0, 0, 0, P, None, None))    # s < k
    _err(L, L.hpc_seed_kmeanspp(None, 100, 4, P, 10, 3, 3, 0, 0, 0, P, None, None))
    _err(L, L.hpc_assign_sse(P, 0, 4, P, 3, 0, None, None, P, None))
    _err(L, L.hpc_assign_sse(P, 10, 4, P, 0, 0, None, None, P, None))
    _err(L, L.hpc_assign_sse(P, 10, 4, P, 3, 0, None, None, None, None))
    _err(L, L.hpc_assign_sse(P, 10, 4, P, 3, 9, None, None, P, None))
    _err(L, L.hpc_draw_sample(0, 10, 0, 0, P, None))
    _err(L, L.hpc_draw_sample(10, 0, 0, 0, P, None))
    _err(L, L.hpc_draw_samples(10, _desc((5, 0, 10, 3)), 1, P, 10, None))
    _err(L, L.hpc_keep_best(P, P, P, P, 0, 3, 4, None, None))
    _err(L, L.hpc_select_best(P, P, 0, 3, 4, P, P, None, None))


def test_binding_refuses_cpu_tensors():
    import torch

    from paper_2311_04517_amd import api

    X = torch.zeros(10, 4)
    with pytest.raises(TypeError):
        api.assign_sse(X, torch.zeros(2, 4))
