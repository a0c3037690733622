"""GPU vs oracle parity of every call of the online step, through the C ABI."""
import numpy as np
import pytest

from synth import random_saturation
from oracle.online import reduced_system, solve_reduced, online_step, DIRECT, DIRECT_FIT, AFFINE
from oracle.pressure import Mobility, reconstruct_flux
from oracle.transport import saturation_step

from .helpers import (TOL_BLOCK, TOL_PN, TOL_SAT, TOL_FLUX, log, rel_l2, oracle_case, gpu_model,
                      dev, host)

pytestmark = pytest.mark.gpu

CASES = ["tiny2d", "small2d", "small3d", "cfg1"]


@pytest.fixture(scope="module", params=CASES)
def case(request):
    name = request.param
    log(f"[parity] building case {name}")
    p, g, om, off = oracle_case(name)
    gm = gpu_model(p, om, om.profiles)
    log(f"[parity] {name}: N={gm.info['N']} n_sub={gm.info['n_sub']} profiles={gm.info['n_profiles']}")
    yield name, p, g, om, gm
    gm.close()


def _state(p, seed):
    return random_saturation(p, np.random.default_rng(seed))


@pytest.mark.parametrize("mode", [DIRECT, DIRECT_FIT, AFFINE])
def test_reduced_system(case, mode):
    name, p, g, om, gm = case
    s = _state(p, 21)
    log(f"[parity] {name} mode={mode}: assemble")
    gm.assemble(dev(s), mode)
    assert gm.status() == 0
    A_o, f_o = reduced_system(om, s, mode)
    A_g = gm.dense_reduced_matrix()
    _, f_g = gm.reduced_system()
    A_od = A_o.toarray()
    err = np.abs(A_g - A_od).max() / np.abs(A_od).max()
    log(f"[parity] {name} mode={mode}: A err {err:.2e}")
    assert err <= TOL_BLOCK
    assert rel_l2(f_g, f_o) <= TOL_BLOCK
    if mode != DIRECT:
        from oracle.online import lsq_theta
        th_o = lsq_theta(g, p, s, om.profiles)
        th_g = gm.theta()
        fit = lambda th: sum(t * q for t, q in zip(th, om.profiles))
        assert rel_l2(fit(th_g), fit(th_o)) <= 1e-10


@pytest.mark.parametrize("mode", [DIRECT, AFFINE])
def test_reduced_solve(case, mode):
    import torch
    name, p, g, om, gm = case
    s = _state(p, 22)
    gm.assemble(dev(s), mode)
    pN = torch.zeros(gm.info["N"], dtype=torch.float64, device="cuda")
    log(f"[parity] {name} mode={mode}: solve")
    gm.solve(pN)
    assert gm.status() == 0
    A_o, f_o = reduced_system(om, s, mode)
    pN_o = solve_reduced(A_o, f_o)
    err = rel_l2(host(pN), pN_o)
    log(f"[parity] {name} mode={mode}: pN err {err:.2e}")
    assert err <= TOL_PN


def test_flux_and_transport_lockstep(case):
    """Each fine-grid call fed the oracle's own inputs (p_N, s, F)."""
    import torch
    name, p, g, om, gm = case
    s = _state(p, 23)
    out = online_step(om, s, DIRECT)
    flux = torch.zeros(g.nface, dtype=torch.float64, device="cuda")
    ph = torch.zeros(g.r * g.ncell, dtype=torch.float64, device="cuda")
    log(f"[parity] {name}: reconstruct_flux")
    gm.reconstruct_flux(dev(out["pN"]), dev(s), flux, ph)
    assert rel_l2(host(ph), out["ph"]) <= TOL_PN
    ef = rel_l2(host(flux), out["F"])
    log(f"[parity] {name}: flux err {ef:.2e}")
    assert ef <= TOL_FLUX
    s_out = torch.zeros_like(ph)
    flags = torch.zeros(g.ncell, dtype=torch.uint8, device="cuda")
    log(f"[parity] {name}: transport_step")
    gm.transport_step(dev(s), dev(out["F"]), s_out, flags)
    es = rel_l2(host(s_out), out["s"])
    log(f"[parity] {name}: sat err {es:.2e} flags gpu {int(host(flags).sum())} oracle {int(out['flags'].sum())}")
    assert es <= TOL_SAT
    assert np.array_equal(host(flags), out["flags"])


def test_free_running(case):
    """Alg. 3 step 5 repeated on the GPU from s0 = 0 for the configured number
    of steps (at most 20) against the oracle's own run."""
    import torch
    name, p, g, om, gm = case
    nsteps = min(p.n_steps, 20)
    s_o = np.zeros(g.r * g.ncell)
    s_a = torch.zeros(g.r * g.ncell, dtype=torch.float64, device="cuda")
    s_b = torch.zeros_like(s_a)
    pN = torch.zeros(gm.info["N"], dtype=torch.float64, device="cuda")
    flux = torch.zeros(g.nface, dtype=torch.float64, device="cuda")
    log(f"[parity] {name}: free run {nsteps} steps")
    for n in range(nsteps):
        s_o = online_step(om, s_o, DIRECT)["s"]
        gm.assemble(s_a, DIRECT)
        gm.solve(pN)
        gm.reconstruct_flux(pN, s_a, flux)
        gm.transport_step(s_a, flux, s_b)
        s_a, s_b = s_b, s_a
    assert gm.status() == 0
    err = rel_l2(host(s_a), s_o)
    log(f"[parity] {name}: free-run sat err {err:.2e}")
    assert err <= TOL_SAT


def test_solve_before_assemble_is_state_error():
    import torch
    from paper_1405_2810_amd.lrbms import LrbmsError
    p, g, om, off = oracle_case("tiny2d", with_profiles=False)
    gm = gpu_model(p, om)
    pN = torch.zeros(gm.info["N"], dtype=torch.float64, device="cuda")
    with pytest.raises(LrbmsError) as ei:
        gm.solve(pN)
    assert ei.value.code == -2
    with pytest.raises(LrbmsError) as ei:
        gm.assemble(dev(np.zeros(g.r * g.ncell)), AFFINE)
    assert ei.value.code == -2
    gm.close()


@pytest.mark.parametrize("name,ne", [("small2d", 20), ("small2d", 40), ("small3d", 20),
                                     ("small3d", 40)])
def test_large_local_bases(name, ne):
    """Local bases of 20 and 40 functions (the wider assembly variants and
    multi-panel fronts): reduced system and reduced solve."""
    import torch
    from .helpers import synthetic_case
    log(f"[parity] large bases {name} N_E={ne}")
    p, g, om = synthetic_case(name, n_snap=ne + 2, cap=ne)
    gm = gpu_model(p, om)
    s = _state(p, 31)
    gm.assemble(dev(s), DIRECT)
    A_o, f_o = reduced_system(om, s, DIRECT)
    A_od = A_o.toarray()
    err = np.abs(gm.dense_reduced_matrix() - A_od).max() / np.abs(A_od).max()
    _, f_g = gm.reduced_system()
    e_f = rel_l2(f_g, f_o)
    log(f"[parity] large bases {name} N_E={ne}: A err {err:.2e} f err {e_f:.2e}")
    assert err <= TOL_BLOCK
    assert e_f <= TOL_BLOCK
    pN = torch.zeros(gm.info["N"], dtype=torch.float64, device="cuda")
    gm.solve(pN)
    assert gm.status() == 0
    e_p = rel_l2(host(pN), solve_reduced(A_o, f_o))
    log(f"[parity] large bases {name} N_E={ne}: pN err {e_p:.2e}")
    assert e_p <= TOL_PN
    gm.close()


@pytest.mark.parametrize("name,ne", [("tiny2d", 6), ("small2d", 20), ("small2d", 60),
                                     ("small3d", 12), ("small3d", 40), ("small3d", 60)])
def test_assembly_variants(name, ne):
    """Both box-assembly variants (four waves with several columns per thread;
    six waves with one (cell, column) item per thread, chunks of 30 cells in
    3D, the contraction padded to a multiple of four rows in 2D at 64
    columns) against the oracle's reduced system, and against each other."""
    from .helpers import synthetic_case
    p, g, om = synthetic_case(name, n_snap=ne + 2, cap=ne)
    gm = gpu_model(p, om)
    try:
        s = _state(p, 41)
        A_o, f_o = reduced_system(om, s, DIRECT)
        A_od = A_o.toarray()
        got = []
        for v in (0, 1):
            gm.set_assembly_variant(v)
            gm.assemble(dev(s), DIRECT)
            assert gm.status() == 0
            A_g = gm.dense_reduced_matrix()
            _, f_g = gm.reduced_system()
            err = np.abs(A_g - A_od).max() / np.abs(A_od).max()
            log(f"[parity] assembly variant {v} {name} N_E={ne}: A err {err:.2e} "
                f"f err {rel_l2(f_g, f_o):.2e}")
            assert err <= TOL_BLOCK
            assert rel_l2(f_g, f_o) <= TOL_BLOCK
            got.append((A_g, f_g))
        assert np.abs(got[0][0] - got[1][0]).max() <= 1e-13 * np.abs(A_od).max()
    finally:
        gm.close()
