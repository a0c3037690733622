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


def test_null_out_pointer(L):
    lib = L.lib()
    assert lib.lrbms_model_create(None, None, None, 0, None, None) == -1
    assert b"NULL" in lib.lrbms_last_error()
