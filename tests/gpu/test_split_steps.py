"""Split launches of the reduced solver, forced on small problems through
the environment when the model is created (large workloads split only their
largest fronts):
* panel steps split into a rows-only launch and the trailing updates (which
  read both L tiles from the L store) against the fused steps: the same
  arithmetic on the same values, so p_N must agree bit for bit
  (LRBMS_STEP_SPLIT_MIN=1);
* the backward product L_US^T x_U split over workgroups of 64 U rows
  (LRBMS_BW_SPLIT_MIN=1): other summation order, so p_N is checked against
  the oracle's reduced solve."""
import os

import numpy as np
import pytest

from synth import make_problem, random_saturation, smooth_fields

from .helpers import log

pytestmark = pytest.mark.gpu


def _with_env(var, value, make):
    old = os.environ.get(var)
    os.environ[var] = str(value)
    try:
        return make()
    finally:
        if old is None:
            del os.environ[var]
        else:
            os.environ[var] = old


def _model(L, p, snaps, split_min):
    return _with_env("LRBMS_STEP_SPLIT_MIN", split_min,
                     lambda: L.Model.from_snapshots(p, snaps, ne_cap=p.ne_cap, unit_functions=True))


@pytest.mark.parametrize("name", ["tiny2d", "small2d", "small3d", "cfg1", "cfg2"])
def test_split_steps_equal_fused(name):
    import torch
    from paper_1405_2810_amd import lrbms as L
    p = make_problem(name)
    snaps = smooth_fields(p, p.ne_cap + 2, np.random.default_rng(31))
    fused = _model(L, p, snaps, 1 << 30)
    split = _model(L, p, snaps, 1)
    try:
        for seed in (1, 2):
            s = torch.tensor(random_saturation(p, np.random.default_rng(seed)),
                             dtype=torch.float64, device="cuda")
            out = []
            for m in (fused, split):
                pN = torch.zeros(m.info["N"], dtype=torch.float64, device="cuda")
                m.assemble(s)
                m.solve(pN)
                out.append(pN)
            torch.cuda.synchronize()
            assert fused.status() == 0 and split.status() == 0
            log(f"[split] {name} seed {seed}: N={fused.info['N']} max |diff| "
                f"{(out[0] - out[1]).abs().max().item():.3e}")
            assert torch.equal(out[0], out[1])
    finally:
        fused.close()
        split.close()


@pytest.mark.parametrize("name", ["small2d", "small3d", "cfg1"])
def test_split_backward_product(name):
    import torch
    from paper_1405_2810_amd import lrbms as L
    from oracle.online import reduced_system, solve_reduced, DIRECT
    from .helpers import TOL_PN, rel_l2, oracle_case, gpu_model, dev, host
    p, g, om, _ = oracle_case(name)
    gm = _with_env("LRBMS_BW_SPLIT_MIN", 1, lambda: gpu_model(p, om))
    try:
        for seed in (3, 4):
            s = random_saturation(p, np.random.default_rng(seed))
            pN = torch.zeros(gm.info["N"], dtype=torch.float64, device="cuda")
            gm.assemble(dev(s), L.DIRECT)
            gm.solve(pN)
            assert gm.status() == 0
            A, f = reduced_system(om, s, DIRECT)
            err = rel_l2(host(pN), solve_reduced(A, f))
            log(f"[split] {name} backward product split, seed {seed}: p_N err {err:.2e}")
            assert err <= TOL_PN
    finally:
        gm.close()


def test_set_solver_shapes():
    """lrbms_model_set_solver_shapes installs the plan of given shapes: each
    plan's p_N meets the oracle's reduced solve, setting the same shapes
    again reproduces p_N bit for bit, and shapes out of range are refused."""
    import torch
    from paper_1405_2810_amd import lrbms as L
    from oracle.online import reduced_system, solve_reduced, DIRECT
    from .helpers import TOL_PN, rel_l2, oracle_case, gpu_model, dev, host
    p, g, om, _ = oracle_case("small3d")
    gm = gpu_model(p, om)
    try:
        s = random_saturation(p, np.random.default_rng(7))
        gm.assemble(dev(s), L.DIRECT)
        ref = solve_reduced(*reduced_system(om, s, DIRECT))
        first = {}
        for shapes in [(1, 0, 0), (2, 1, 1), (8, 256, 0), (1, 0, 0)]:
            gm.set_solver_shapes(*shapes)
            pN = torch.zeros(gm.info["N"], dtype=torch.float64, device="cuda")
            gm.solve(pN)
            assert gm.status() == 0
            err = rel_l2(host(pN), ref)
            log(f"[shapes] {shapes}: p_N err {err:.2e}")
            assert err <= TOL_PN
            if shapes in first:
                assert torch.equal(first[shapes], pN)
            first[shapes] = pN
        for bad in [(0, 0, 0), (65, 0, 0), (2, -1, 0), (2, 0, -1)]:
            with pytest.raises(L.LrbmsError) as ei:
                gm.set_solver_shapes(*bad)
            assert ei.value.code == -1
    finally:
        gm.close()
