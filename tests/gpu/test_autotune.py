"""The solver autotuner (lrbms_model_autotune): it times every candidate
shape of the reduced solver on the device and keeps the fastest; the
model's reduced pressure stays the oracle's (another elimination order
changes only the rounding)."""
import numpy as np
import pytest

from synth import random_saturation
from oracle.online import reduced_system, solve_reduced, DIRECT

from .helpers import TOL_PN, log, rel_l2, oracle_case, gpu_model, dev, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["small2d", "small3d", "cfg1"])
def test_autotune_keeps_parity(name):
    import torch
    from paper_1405_2810_amd import lrbms as L
    p, g, om, _ = oracle_case(name)
    gm = gpu_model(p, om, om.profiles)
    try:
        s = random_saturation(p, np.random.default_rng(7))
        rep = gm.autotune(dev(s), reps=3)
        log(f"[autotune] {name}: {rep}")
        assert rep["n_candidates"] >= 5
        assert rep["leaf_max"] in (1, 2, 4, 8, 16)
        assert rep["split_min"] in (0, 256, 1024)
        assert rep["bw_split_min"] in (0, 1 << 12, 1 << 14, 1 << 16, 1 << 18)
        assert 0.0 < rep["us_per_solve"] <= rep["us_before"] * (1 + 1e-12)
        for seed in (8, 9):
            s = random_saturation(p, np.random.default_rng(seed))
            pN = torch.zeros(gm.info["N"], dtype=torch.float64, device="cuda")
            gm.assemble(dev(s), L.DIRECT)
            gm.solve(pN)
            assert gm.status() == 0
            A, f = reduced_system(om, s, DIRECT)
            err = rel_l2(host(pN), solve_reduced(A, f))
            log(f"[autotune] {name} seed {seed}: p_N err {err:.2e}")
            assert err <= TOL_PN
    finally:
        gm.close()


def test_autotune_arguments():
    from paper_1405_2810_amd import lrbms as L
    p, g, om, _ = oracle_case("tiny2d")
    gm = gpu_model(p, om)
    try:
        with pytest.raises(L.LrbmsError) as ei:
            gm.autotune(None)
        assert ei.value.code == -1
        B = L.Batch([gm])
        with pytest.raises(L.LrbmsError) as ei:
            gm.autotune(dev(random_saturation(p, np.random.default_rng(1))))
        assert ei.value.code == -2
        B.close()
    finally:
        gm.close()
