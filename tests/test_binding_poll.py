"""Server.poll keeps the finished-request records that the library handed
over in a call that then reports an error, and returns them first on the
next call (binding logic only: the library is replaced by a stand-in, no
device is used)."""
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
