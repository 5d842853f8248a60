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
    _err(L, call(prec=3))
    _err(L, call(prec=-1))
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


def test_plan_validation(L):
    h = ct.c_void_p()
    good = _desc((0, 0, 10, 3))
    _err(L, L.hpc_plan_create(4, good, 1, 10, 12, 0, None))                  # NULL out
    _err(L, L.hpc_plan_create(0, good, 1, 10, 12, 0, ct.byref(h)))           # d = 0
    _err(L, L.hpc_plan_create(4, good, 1, 10, 12, 5, ct.byref(h)))           # precision
    _err(L, L.hpc_plan_create(4, _desc((0, 0, 2, 3)), 1, 10, 12, 0, ct.byref(h)))   # s < k
    _err(L, L.hpc_plan_create(4, _desc((5, 0, 10, 3)), 1, 10, 12, 0, ct.byref(h)))  # idx range
    _err(L, L.hpc_plan_create(4, good, 0, 10, 12, 0, ct.byref(h)))           # no samples
    assert h.value is None
    t = _lib.Tune(0, 0, 0, 0, 0, 0)
    _err(L, L.hpc_plan_set_tune(None, ct.byref(t)))
    _err(L, L.hpc_plan_get_tune(None, ct.byref(t)))
    _err(L, L.hpc_plan_replay(None, 1, None))
    _err(L, L.hpc_plan_lloyd(None, P, 10, P, P, 3, 0.0, P, P, None, None))
    _err(L, L.hpc_plan_round(None, P, 10, P, P, P, P, 3, 0.0, P, P, 0, None))
    _err(L, L.hpc_plan_capture_round(None, P, 10, P, P, P, P, 3, 0.0, P, P, 0))
    _err(L, L.hpc_plan_reset_ids(None, None))
    buf = ct.create_string_buffer(8)
    _err(L, L.hpc_plan_tune_key(None, buf, 8))
    assert L.hpc_plan_destroy(None) == _lib.HPC_OK


def test_tuning_cache_roundtrip(tmp_path):
    from paper_2311_04517_amd import tuning

    p = str(tmp_path / "sub" / "tune.json")
    assert tuning.load(p) == {}
    tuning.store({"gfx950|d32|p0|n2^10|k2^5|s2^14": {"wg_per_cu": 2, "copies": 4, "order": 0,
                                                      "ms": 3.1}}, p)
    db = tuning.load(p)
    assert db["gfx950|d32|p0|n2^10|k2^5|s2^14"]["copies"] == 4

    class FakePlan:
        def tune_key(self):
            return "gfx950|d32|p0|n2^10|k2^5|s2^14"

        def set_tune(self, **cfg):
            self.cfg = cfg

    fp = FakePlan()
    cfg, ms = tuning.tuned(fp, None, None, None, path=p)
    # an entry written before the seeding team size and the parts per
    # sample were tuned reads them as 0 (automatic)
    assert ms is None and fp.cfg == {"wg_per_cu": 2, "copies": 4, "order": 0, "seed_team": 0,
                                  "seed_inflight": 0, "parts": 0}


def test_plan_draw_advance_validation(L):
    _err(L, L.hpc_plan_draw(None, 10, P, None))
    _err(L, L.hpc_plan_advance(None, 1, None))


def test_setenc_validation(L):
    h = ct.c_void_p()
    _err(L, L.hpc_setenc_create(33, 25, 1024, 8, 0, ct.byref(h)))   # d > 32
    _err(L, L.hpc_setenc_create(32, 65, 1024, 8, 0, ct.byref(h)))   # k > 64
    _err(L, L.hpc_setenc_create(32, 25, 8, 8, 0, ct.byref(h)))      # n_enc < 16
    _err(L, L.hpc_setenc_create(32, 25, 1024, 0, 0, ct.byref(h)))   # max_batch < 1
    _err(L, L.hpc_setenc_create(32, 25, 1024, 8, 0, None))
    assert h.value is None
    n = ct.c_int64()
    _err(L, L.hpc_setenc_param_count(None, ct.byref(n)))
    _err(L, L.hpc_setenc_get_params(None, 0, P))
    _err(L, L.hpc_setenc_propose(None, P, 10, P, 10, _desc((0, 0, 10, 3)), 1, P, 12, None))
    _err(L, L.hpc_setenc_grad(None, P, 10, P, 10, _desc((0, 0, 10, 3)), 1, P, 12, None, None))
    _err(L, L.hpc_setenc_adam(None, ct.c_float(1e-3), None))
    _err(L, L.hpc_learned_seed(None, P, 10, P, 10, _desc((0, 0, 10, 3)), 1, P, P, 12, 0, P, P,
                               None, None))
    assert L.hpc_setenc_destroy(None) == _lib.HPC_OK
