"""Online failure detection, forced from the host with inputs that every
kernel still processes normally: a saturation state holding a NaN (the
transport step's output is not finite: LRBMS_E_NONFINITE), a time step far
above the CFL bound of the fluxes (LRBMS_W_CFL, a positive warning), and a
clean step (0).  With checks on, the online call that met the condition
returns it; lrbms_model_status returns it too, and keeps it."""
import numpy as np
import pytest

from synth import random_saturation
from oracle.online import DIRECT

from .helpers import log, synthetic_case, gpu_model, dev

pytestmark = pytest.mark.gpu


def _step(gm, s, checks):
    import torch
    gm.set_checks(checks)
    pN = torch.zeros(gm.info["N"], dtype=torch.float64, device="cuda")
    flux = torch.zeros(gm.info["nface"], dtype=torch.float64, device="cuda")
    out = torch.zeros_like(s)
    rcs = [gm.assemble(s, DIRECT), gm.solve(pN), gm.reconstruct_flux(pN, s, flux)]
    rcs.append(gm.transport_step(s, flux, out))
    return rcs, flux, out


def test_clean_step_reports_nothing():
    p, g, om = synthetic_case("tiny2d")
    gm = gpu_model(p, om)
    s = dev(random_saturation(p, np.random.default_rng(3)))
    rcs, _, _ = _step(gm, s, True)
    log(f"[failure] clean step return codes {rcs}")
    assert rcs == [0, 0, 0, 0]
    assert gm.status() == 0
    gm.close()


def test_nan_state_is_reported():
    import torch
    from paper_1405_2810_amd.lrbms import LrbmsError
    p, g, om = synthetic_case("tiny2d")
    gm = gpu_model(p, om)
    s = random_saturation(p, np.random.default_rng(4))
    gm.set_checks(True)
    good = dev(s)
    pN = torch.zeros(gm.info["N"], dtype=torch.float64, device="cuda")
    flux = torch.zeros(gm.info["nface"], dtype=torch.float64, device="cuda")
    assert gm.assemble(good, DIRECT) == 0
    assert gm.solve(pN) == 0
    assert gm.reconstruct_flux(pN, good, flux) == 0
    bad = s.copy()
    bad[g.ncell + 5] = np.nan           # a slope coefficient of one cell
    out = torch.zeros_like(good)
    with pytest.raises(LrbmsError) as ei:
        gm.transport_step(dev(bad), flux, out)
    log(f"[failure] NaN state: {ei.value}")
    assert ei.value.code == -6
    assert gm.status() == -6
    gm.close()


def test_oversized_time_step_warns():
    p, g, om = synthetic_case("tiny2d")
    gm = gpu_model(p.copy(dt=100.0 * p.dt), om)
    s = dev(random_saturation(p, np.random.default_rng(5)))
    rcs, _, _ = _step(gm, s, True)
    log(f"[failure] dt x 100: return codes {rcs}")
    assert rcs[:3] == [0, 0, 0] and rcs[3] == 1
    assert gm.status() == 1
    gm.close()


def test_checks_off_stays_asynchronous_and_status_reports():
    p, g, om = synthetic_case("tiny2d")
    gm = gpu_model(p.copy(dt=100.0 * p.dt), om)
    s = dev(random_saturation(p, np.random.default_rng(6)))
    rcs, _, _ = _step(gm, s, False)
    assert rcs == [0, 0, 0, 0]
    assert gm.status() == 1
    gm.close()
