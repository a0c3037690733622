"""The C ABI library loads and exports every declared symbol; argument checks
that happen before any device work (no GPU needed)."""
import ctypes as C

import numpy as np
import pytest

from synth import make_problem


@pytest.fixture(scope="module")
def L():
    from paper_1405_2810_amd import lrbms
    return lrbms


def test_exports_every_declared_symbol(L):
    lib = L.lib()
    names = L.header_functions()
    assert len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


def test_invalid_problem_rejected_before_device_work(L):
    p = make_problem("tiny2d")
    bad = p.copy(dt=-1.0)
    with pytest.raises(L.LrbmsError) as ei:
        L.Model.create(bad, [1] * 4, np.zeros(3 * 64))
    assert ei.value.code == -1 and "dt" in str(ei.value)
    bad = p.copy()
    bad.cuts[0] = np.array([0, 5, 3], dtype=np.int32)
    with pytest.raises(L.LrbmsError) as ei:
        L.Model.create(bad, [1] * 4, np.zeros(3 * 64))
    assert ei.value.code == -1
    # the problem statement carries gravity; the library solves the case
    # without it and says so instead of ignoring a non-zero vector
    bad = p.copy(grav=(0.0, -9.81, 0.0))
    with pytest.raises(L.LrbmsError) as ei:
        L.Model.create(bad, [1] * 4, np.zeros(3 * 64))
    assert ei.value.code == -1 and "gravity" in str(ei.value)
    bad = p.copy(dens_w=float("nan"))
    with pytest.raises(L.LrbmsError) as ei:
        L.Model.create(bad, [1] * 4, np.zeros(3 * 64))
    assert ei.value.code == -1


def test_null_out_pointer(L):
    lib = L.lib()
    assert lib.lrbms_model_create(None, None, None, 0, None, None) == -1
    assert b"NULL" in lib.lrbms_last_error()


def test_offline_arguments_checked_before_device_work(L):
    p = make_problem("tiny2d")
    mu = np.eye(4)
    cases = [dict(mu=np.eye(2), ne_cap=4, horizon=1.0),          # M < 3
             dict(mu=mu, ne_cap=0, horizon=1.0),                 # cap
             dict(mu=mu, ne_cap=64, horizon=1.0),
             dict(mu=mu, ne_cap=4, horizon=0.0),                 # horizon
             dict(mu=mu, ne_cap=4, horizon=1.0, pcg_rtol=0.0),
             dict(mu=mu, ne_cap=4, horizon=1.0, tof_maxit=0),
             dict(mu=np.full((2, 4), np.nan), ne_cap=4, horizon=1.0)]
    for kw in cases:
        with pytest.raises(L.LrbmsError) as ei:
            L.Model.build_offline(p, **kw)
        assert ei.value.code == -1, kw
    lib = L.lib()
    pc = L.ProblemC(p)
    opts = L.OfflineOpts_C(M=4, n_train=4, ne_cap=4, unit_functions=1, horizon=1.0,
                           pcg_rtol=1e-12, pcg_maxit=10, tof_tol=0.0, tof_maxit=10,
                           keep_profiles=1)
    h = C.c_void_p()
    assert lib.lrbms_build_offline_bases(pc.ref(), C.byref(opts), None, C.byref(h), None) == -1


def test_fine_solver_arguments_checked_before_device_work(L):
    p = make_problem("tiny2d")
    with pytest.raises(L.LrbmsError) as ei:
        L.fine_pressure(p, None, None)
    assert ei.value.code == -1
    buf = np.zeros(3 * 64)   # any non-NULL address: rejected before use
    for kw in (dict(kind=2), dict(rtol=0.0), dict(maxit=0)):
        with pytest.raises(L.LrbmsError) as ei:
            L.fine_pressure(p, buf, buf, **kw)
        assert ei.value.code == -1, kw
    with pytest.raises(L.LrbmsError) as ei:
        L.time_of_flight(p, buf, buf, tol=-1.0)
    assert ei.value.code == -1
    with pytest.raises(L.LrbmsError) as ei:
        L.time_of_flight(p, None, buf)
    assert ei.value.code == -1


def test_batch_and_server_arguments_checked_before_device_work(L):
    lib = L.lib()
    h = C.c_void_p()
    assert lib.lrbms_batch_create(None, 0, 0, 0, C.byref(h)) == -1
    models = (C.c_void_p * 1)(None)
    assert lib.lrbms_batch_create(models, 1, 0, 0, C.byref(h)) == -1
    assert lib.lrbms_batch_step(None, None, None, None) == -1
    assert lib.lrbms_batch_buffers(None, 0, None, None) == -1
    for budget, slots, mode in ((0, 4, 0), (1 << 30, 0, 0), (1 << 30, 65, 0), (1 << 30, 4, 9)):
        assert lib.lrbms_server_create(budget, slots, mode, C.byref(h)) == -1
    sid = C.c_int32()
    assert lib.lrbms_server_attach(None, None, None, C.byref(sid)) == -1
    assert lib.lrbms_server_submit(None, 0, 1) == -1
    n = C.c_int32()
    assert lib.lrbms_server_poll(None, None, None, None, 0, C.byref(n)) == -1
    assert lib.lrbms_server_drain(None) == -1
    assert lib.lrbms_server_detach(None, 0) == -1
    assert lib.lrbms_server_info(None, None) == -1
    lib.lrbms_batch_destroy(None)
    lib.lrbms_server_destroy(None)
    assert lib.lrbms_model_autotune(None, None, 1, None) == -1
