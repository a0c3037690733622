"""Split panel steps of the reduced solver (rows-only launch, then the
trailing updates reading both L tiles from the L store) against the fused
steps: the same arithmetic on the same values, so p_N must agree bit for
bit.  Splitting is forced for every step by LRBMS_STEP_SPLIT_MIN=1 when the
model is created (large workloads split only their largest steps)."""
import os

import numpy as np
import pytest

from synth import make_problem, random_saturation, smooth_fields

from .helpers import log

pytestmark = pytest.mark.gpu


def _model(L, p, snaps, split_min):
    old = os.environ.get("LRBMS_STEP_SPLIT_MIN")
    os.environ["LRBMS_STEP_SPLIT_MIN"] = str(split_min)
    try:
        return L.Model.from_snapshots(p, snaps, ne_cap=p.ne_cap, unit_functions=True)
    finally:
        if old is None:
            del os.environ["LRBMS_STEP_SPLIT_MIN"]
        else:
            os.environ["LRBMS_STEP_SPLIT_MIN"] = old


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
