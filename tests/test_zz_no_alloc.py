"""lrbms_time_of_flight_noalloc (work buffers in the library's fixed scratch
array) against lrbms_time_of_flight (work buffers allocated per call), on two
calls in a row, the second with a smaller problem: the same kernels in the
same order, so tau must agree bit for bit, and both within the oracle's
1e-10 of the time of flight (eq. timeOfFlight)."""
import numpy as np
import pytest

from synth import make_problem
from oracle.fem import Grid
from oracle.tof import time_of_flight as oracle_tof
from oracle.offline import initial_flow

from tests.gpu.helpers import log, rel_l2, dev, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("names", [("cfg1", "small2d"), ("small3d", "tiny2d")])
def test_noalloc_time_of_flight_matches_allocating_one(names):
    from paper_1405_2810_amd import lrbms as L
    for name in names:
        p = make_problem(name)
        g = Grid(p)
        _, F0 = initial_flow(g, p)
        ref = dev(np.zeros(g.r * g.ncell))
        out = dev(np.full(g.r * g.ncell, np.nan))
        s_ref = L.time_of_flight(p, dev(F0), ref, tol=0.0)
        s_out = L.time_of_flight(p, dev(F0), out, tol=0.0, noalloc=True)
        a, b = host(ref), host(out)
        err_o = rel_l2(b, oracle_tof(g, p, F0))
        log(f"[noalloc] {name}: sweeps {s_ref} / {s_out}, max |diff| {np.abs(a - b).max():.1e}, "
            f"vs oracle {err_o:.2e}")
        assert s_out == s_ref
        assert np.array_equal(a, b)
        assert err_o <= 1e-10


def test_noalloc_rejects_a_problem_beyond_its_scratch():
    from paper_1405_2810_amd import lrbms as L
    p = make_problem("cfg3")
    out = dev(np.zeros((p.dim + 1) * p.ncell))
    with pytest.raises(L.LrbmsError) as ei:
        L.time_of_flight(p, dev(np.zeros(len(p.bc_type))), out, noalloc=True)
    assert ei.value.code == -1
