"""The paper's 2D benchmark shape (Sec. 6): [0,300] x [0,60] m in 400 x 160
cells, linear relative permeabilities, the printed viscosities, water
entering on the left (Dirichlet p = 10 and s = 1 on Gamma_s,d), outward flux
3e-4 on the right, no flow on top and bottom, no sources; seeded
permeability and porosity stand in for the paper's fields (figure
placeholders), 8 x 2 boxes.

* Alg. 1 (the fine scheme) on the GPU against the oracle's: fine pressure,
  fluxes, saturation and limiter flags of two steps from s0 = 0.
* Alg. 2 without the greedy selection on the oracle (time of flight,
  mobility profiles, snapshots, local Gram-Schmidt), then the online step
  of Alg. 3 with those bases on the GPU against the oracle's: three free
  steps from s0 = 0 (p_N, saturation, no warning: their CFL numbers stay
  below 1/2), then one step from a seeded saturation in lockstep (reduced
  system, p_N, fluxes, saturation, flags, and the CFL warning exactly when
  the oracle's fluxes give a CFL number above 1/2)."""
import numpy as np
import pytest

from synth import make_problem, random_saturation, training_params
from oracle.fem import Grid
from oracle.offline import build_offline
from oracle.online import Model as OModel, reduced_system, solve_reduced, online_step, DIRECT
from oracle.schemes import fine_impes

from .helpers import (TOL_BLOCK, TOL_PN, TOL_SAT, TOL_FLUX, cfl_number, log, rel_l2, gpu_model,
                      dev, host)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def paper():
    p = make_problem("paper")
    return p, Grid(p)


def test_paper_case_fine_scheme(paper):
    """Two steps of Alg. 1: GPU (multigrid CG to 1e-13) against the oracle
    (sparse direct solve)."""
    import torch
    from paper_1405_2810_amd.lrbms import Fine
    p, g = paper
    _, hist = fine_impes(g, p, np.zeros(g.r * g.ncell), 2)
    fine = Fine(p)
    s_a = torch.zeros(g.r * g.ncell, dtype=torch.float64, device="cuda")
    s_b, ph = torch.zeros_like(s_a), torch.zeros_like(s_a)
    flux = torch.zeros(g.nface, dtype=torch.float64, device="cuda")
    flags = torch.zeros(g.ncell, dtype=torch.uint8, device="cuda")
    for n in range(2):
        it, rr = fine.step(s_a, ph, flux, s_b, flags, warm=n > 0)
        e_p, e_f = rel_l2(host(ph), hist[n]["p"]), rel_l2(host(flux), hist[n]["F"])
        e_s = rel_l2(host(s_b), hist[n]["s"])
        log(f"[paper] fine step {n}: CG {it} it (relres {rr:.1e}); p err {e_p:.2e} flux err "
            f"{e_f:.2e} sat err {e_s:.2e} flags {int(host(flags).sum())}/{int(hist[n]['flags'].sum())}")
        assert e_p <= 1e-9
        assert e_f <= 1e-9
        assert e_s <= TOL_SAT
        assert np.array_equal(host(flags), hist[n]["flags"])
        s_a, s_b = s_b, s_a
    fine.close()


def test_paper_case_online_step(paper):
    import torch
    p, g = paper
    params = training_params(p.M, p.n_train, np.random.default_rng(p.seed))
    off = build_offline(g, p, params)
    om = OModel(p, off["basis"].phis, None)
    gm = gpu_model(p, om)
    log(f"[paper] offline bases: N={gm.info['N']} (N_E <= {p.ne_cap}), "
        f"profiles kept {len(off['keep'])}")
    pN = torch.zeros(gm.info["N"], dtype=torch.float64, device="cuda")
    flux = torch.zeros(g.nface, dtype=torch.float64, device="cuda")
    s_o = np.zeros(g.r * g.ncell)
    s_a = torch.zeros(g.r * g.ncell, dtype=torch.float64, device="cuda")
    s_b = torch.zeros_like(s_a)
    cfl = 0.0
    for n in range(3):
        o = online_step(om, s_o, DIRECT)
        s_o = o["s"]
        cfl = max(cfl, cfl_number(p, o["F"]))
        gm.assemble(s_a, DIRECT)
        gm.solve(pN)
        e_p = rel_l2(host(pN), o["pN"])
        gm.reconstruct_flux(pN, s_a, flux)
        gm.transport_step(s_a, flux, s_b)
        s_a, s_b = s_b, s_a
        log(f"[paper] online step {n}: pN err {e_p:.2e} sat err {rel_l2(host(s_a), s_o):.2e} "
            f"CFL {cfl_number(p, o['F']):.3f}")
        assert e_p <= TOL_PN
    assert cfl < 0.49 and gm.status() == 0
    assert rel_l2(host(s_a), s_o) <= TOL_SAT
    s = random_saturation(p, np.random.default_rng(3), lo=0.0, hi=0.8)
    gm.assemble(dev(s), DIRECT)
    A_o, f_o = reduced_system(om, s, DIRECT)
    A_od = A_o.toarray()
    err = np.abs(gm.dense_reduced_matrix() - A_od).max() / np.abs(A_od).max()
    _, f_g = gm.reduced_system()
    gm.solve(pN)
    e_p = rel_l2(host(pN), solve_reduced(A_o, f_o))
    log(f"[paper] reduced system: A err {err:.2e} f err {rel_l2(f_g, f_o):.2e} pN err {e_p:.2e}")
    assert err <= TOL_BLOCK and rel_l2(f_g, f_o) <= TOL_BLOCK and e_p <= TOL_PN
    out = online_step(om, s, DIRECT)
    gm.reconstruct_flux(dev(out["pN"]), dev(s), flux)
    s_out = torch.zeros(g.r * g.ncell, dtype=torch.float64, device="cuda")
    flags = torch.zeros(g.ncell, dtype=torch.uint8, device="cuda")
    gm.transport_step(dev(s), dev(out["F"]), s_out, flags)
    ef, es = rel_l2(host(flux), out["F"]), rel_l2(host(s_out), out["s"])
    log(f"[paper] online step lockstep: flux err {ef:.2e} sat err {es:.2e} "
        f"flags {int(host(flags).sum())}/{int(out['flags'].sum())}")
    assert ef <= TOL_FLUX and es <= TOL_SAT
    assert np.array_equal(host(flags), out["flags"])
    cfl = cfl_number(p, out["F"])
    log(f"[paper] lockstep CFL {cfl:.3f}, status {gm.status()}")
    if abs(cfl - 0.5) > 5e-3:
        assert gm.status() == (1 if cfl > 0.5 else 0)   # LRBMS_W_CFL = 1
    gm.close()
