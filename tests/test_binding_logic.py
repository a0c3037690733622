"""Logic of the Python binding with the library replaced by a stand-in (no
device is used): Server.poll keeps the finished-request records that the
library handed over in a call that then reports an error, and returns them
first on the next call; a model held by an open batch or server is not
closed (the library would refuse to destroy it and the handle would be
lost), and closes once the batch is closed or the model detached."""
import ctypes as C

import numpy as np
import pytest


class _FakeLib:
    """lrbms_server_poll: first call hands over two records and fails with
    E_OOM, second call hands over one record and succeeds."""

    def __init__(self):
        self.calls = 0

    def lrbms_server_poll(self, h, ids, lat, st, cap, n_done):
        batches = [([11, 12], -3), ([13], 0)]
        recs, rc = batches[self.calls]
        self.calls += 1
        a = np.ctypeslib.as_array((C.c_uint64 * cap).from_address(ids))
        b = np.ctypeslib.as_array((C.c_double * cap).from_address(lat))
        c = np.ctypeslib.as_array((C.c_int32 * cap).from_address(st))
        for k, r in enumerate(recs):
            a[k], b[k], c[k] = r, 0.5 * r, 0
        C.cast(n_done, C.POINTER(C.c_int32))[0] = len(recs)
        return rc

    def lrbms_last_error(self):
        return b"host allocation failed"


def test_poll_keeps_records_across_an_error(monkeypatch):
    from paper_1405_2810_amd import lrbms
    fake = _FakeLib()
    monkeypatch.setattr(lrbms, "lib", lambda: fake)
    S = object.__new__(lrbms.Server)
    S._carry, S._h = [], None
    with pytest.raises(lrbms.LrbmsError) as ei:
        S.poll(cap=8)
    assert ei.value.code == -3
    got = S.poll(cap=8)
    assert [g[0] for g in got] == [11, 12, 13]
    assert [g[1] for g in got] == [5.5, 6.0, 6.5]
    assert fake.calls == 2


class _FakeOwnerLib:
    def __init__(self):
        self.destroyed = []

    def lrbms_batch_create(self, arr, n, mode, flags, out):
        C.cast(out, C.POINTER(C.c_void_p))[0] = 1234
        return 0

    def lrbms_batch_destroy(self, h):
        self.destroyed.append("batch")

    def lrbms_server_attach(self, h, m, sat, sid):
        C.cast(sid, C.POINTER(C.c_int32))[0] = 0
        return 0

    def lrbms_server_detach(self, h, sim):
        return 0

    def lrbms_server_destroy(self, h):
        self.destroyed.append("server")

    def lrbms_model_destroy(self, h):
        self.destroyed.append(h)

    def lrbms_last_error(self):
        return b""


class _FakeCudaTensor:
    """Stands in for a GPU tensor (is_cuda) of a given dtype, layout and size."""

    def __init__(self, dtype, n, contiguous=True):
        self.dtype, self._n, self._c, self.is_cuda = dtype, n, contiguous, True

    def numel(self):
        return self._n

    def is_contiguous(self):
        return self._c

    def data_ptr(self):
        return 4096


def _fake_model(L, h):
    m = object.__new__(L.Model)
    m._h = h
    return m


def test_model_of_an_open_batch_or_server_is_not_closed(monkeypatch):
    from paper_1405_2810_amd import lrbms
    fake = _FakeOwnerLib()
    monkeypatch.setattr(lrbms, "lib", lambda: fake)
    a, b = _fake_model(lrbms, 7), _fake_model(lrbms, 8)
    B = lrbms.Batch([a, b])
    with pytest.raises(lrbms.LrbmsError) as ei:
        a.close()
    assert ei.value.code == -2 and a._h == 7 and fake.destroyed == []
    B.close()
    a.close()
    assert fake.destroyed == ["batch", 7] and a._h is None
    S = object.__new__(lrbms.Server)
    S._carry, S._sims, S._states, S._h = [], {}, {}, 99
    state = _FakeCudaTensor(np.float64, 48)
    monkeypatch.setattr(lrbms, "_dev", lambda t, dtype, n, name, optional=False: 4096)
    b.info = dict(r=3, ncell=16)
    sid = S.attach(b, state)
    assert S._states[sid] is state
    with pytest.raises(lrbms.LrbmsError):
        b.close()
    S.detach(sid)
    b.close()
    assert fake.destroyed == ["batch", 7, 8]
    c = _fake_model(lrbms, 9)
    c.info = dict(r=3, ncell=16)
    S.attach(c, state)
    S.close()
    c.close()
    assert fake.destroyed == ["batch", 7, 8, "server", 9]


def test_device_buffers_are_checked_before_the_library(monkeypatch):
    """The online calls accept only contiguous GPU tensors of the expected
    dtype and size: a host array, a CPU tensor, a wrong dtype, a strided
    view or a short tensor raises E_ARG before anything reaches the
    library."""
    import torch
    from paper_1405_2810_amd import lrbms

    class _NoLib:
        def __getattr__(self, name):
            def call(*a):
                raise AssertionError(f"{name} reached the library")
            return call

    monkeypatch.setattr(lrbms, "lib", lambda: _NoLib())
    m = object.__new__(lrbms.Model)
    m._h = None
    m.info = dict(r=3, ncell=16, N=8, nface=40)
    for bad in (np.zeros(48), torch.zeros(48, dtype=torch.float64), None):
        with pytest.raises(lrbms.LrbmsError) as ei:
            m.assemble(bad)
        assert ei.value.code == -1
    with pytest.raises(lrbms.LrbmsError):
        m.solve(torch.zeros(8, dtype=torch.float32))
    assert lrbms._dev(None, "float64", 4, "ph", optional=True) == 0

    _FakeCuda = _FakeCudaTensor
    monkeypatch.setattr(torch, "Tensor", _FakeCuda)
    assert lrbms._dev(_FakeCuda(torch.float64, 48), "float64", 48, "sat") == 4096
    for bad in (_FakeCuda(torch.float32, 48), _FakeCuda(torch.float64, 47),
                _FakeCuda(torch.float64, 48, contiguous=False)):
        with pytest.raises(lrbms.LrbmsError) as ei:
            lrbms._dev(bad, "float64", 48, "sat")
        assert ei.value.code == -1
    assert lrbms._dev(_FakeCuda(torch.uint8, 16), "uint8", 16, "flags") == 4096
