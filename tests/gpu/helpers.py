"""Shared set-up of the GPU parity tests: the oracle builds the reduced model
(bases, profiles) from the seeded problem; the same inputs go to the HIP
library through the C ABI; every comparison is GPU vs oracle."""
import math
import sys

import numpy as np

from synth import make_problem, random_saturation, training_params
from oracle.fem import Grid
from oracle.offline import build_offline, local_bases
from oracle.online import Model as OModel
from oracle.pressure import fine_pressure

TOL_BLOCK = 1e-12   # reduced matrix entries, relative to the largest entry
TOL_PN = 1e-10      # reduced pressure, relative L2
TOL_SAT = 1e-9      # saturation, relative L2
TOL_FLUX = 1e-10    # face fluxes, relative L2


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def cfl_number(p, F):
    """CFL number of an explicit Euler transport step with face fluxes F:
    dt max|f_w'| (slopes over 4096 equal saturation intervals) times a
    cell's outflow over phi |e|, maximised over cells."""
    from synth.problems import face_counts
    s = np.linspace(0.0, 1.0, 4097)
    kw, ko = (s, 1.0 - s) if p.relperm == 0 else (s ** p.corey_w, (1.0 - s) ** p.corey_o)
    fw = (kw / p.visc_w) / (kw / p.visc_w + ko / p.visc_o)
    fmax = np.max(np.abs(np.diff(fw)) * 4096)
    nx, ny, nz = p.n
    fx, fy, _ = face_counts(p.dim, p.n)
    F = np.asarray(F)
    Fx = F[:fx].reshape(nz, ny, nx + 1)
    Fy = F[fx:fx + fy].reshape(nz, ny + 1, nx)
    out = (np.maximum(0, Fx[:, :, 1:]) + np.maximum(0, -Fx[:, :, :-1]) +
           np.maximum(0, Fy[:, 1:, :]) + np.maximum(0, -Fy[:, :-1, :]))
    if p.dim == 3:
        Fz = F[fx + fy:].reshape(nz + 1, ny, nx)
        out = out + np.maximum(0, Fz[1:]) + np.maximum(0, -Fz[:-1])
    vol = float(np.prod(p.h[:p.dim]))
    return float((p.dt * fmax * out.ravel() / (np.asarray(p.poro) * vol)).max())


def oracle_case(name, with_profiles=True, **kw):
    """Problem, oracle model (bases from the oracle's offline stage), the
    flat basis and the kept profiles."""
    p = make_problem(name, **kw)
    g = Grid(p)
    params = training_params(p.M, p.n_train, np.random.default_rng(p.seed))
    off = build_offline(g, p, params)
    profiles = [off["profiles"][k] for k in off["keep"]] if with_profiles else None
    om = OModel(p, off["basis"].phis, profiles)
    return p, g, om, off


def synthetic_case(name, n_snap=6, cap=None, seed=3, **kw):
    """Bases from fine pressures at seeded random saturations (no TOF)."""
    p = make_problem(name, **kw)
    g = Grid(p)
    rng = np.random.default_rng(seed)
    snaps = [fine_pressure(g, p, s=random_saturation(p, rng)) for _ in range(n_snap)]
    phis = local_bases(g, p, snaps, method="gs", cap=cap or p.ne_cap, unit=True)
    return p, g, OModel(p, phis, None)


def gpu_model(p, om, profiles=None):
    from paper_1405_2810_amd.lrbms import Model
    sizes = [phi.shape[0] for phi in om.basis.phis]
    return Model.create(p, sizes, om.basis.flat(), profiles)


def dev(x):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()
