"""Pins of the oracle's mobility law, SWIP assembly, fine solve and velocity
reconstruction against values and identities fixed by the paper and by
the mathematics (not by the oracle itself)."""
import json
import math
import os

import numpy as np
import pytest

from synth import make_problem, random_saturation
from oracle.fem import Grid, mobilities, frac_flow
from oracle.pressure import (Mobility, assemble, rhs, fine_pressure, reconstruct_flux,
                             cell_outflow, solve_spd)
from oracle.brute import brute_assemble

GOLD = os.path.join(os.path.dirname(__file__), "..", "golden", "paper_constants.json")


def test_printed_profile_endpoint():
    """Caption of the wetting mobility profile figure: Lambda_w^M = 765.808 and
    Lambda_w^1 = 0 for the linear law with the printed eta_w (Sec. 6)."""
    g = json.load(open(GOLD))
    p = make_problem("tiny2d")
    p.relperm = 0
    p.visc_w, p.visc_o = g["visc_w"], g["visc_o"]
    lw, lo, lt = mobilities(np.array([0.0, 1.0]), p)
    assert round(lw[1], g["Lambda_w_last_decimals"]) == g["Lambda_w_last"]
    assert lw[0] == g["Lambda_w_first"]
    assert lo[0] == pytest.approx(1.0 / g["visc_o"]) and lo[1] == 0.0


def test_corey_closed_forms():
    p = make_problem("tiny2d")
    s = np.linspace(0, 1, 1001)
    lt = mobilities(s, p)[2]
    # minimum of s^2/eta_w + (1-s)^2/eta_o at s* = eta_w / (eta_w + eta_o)
    sstar = p.visc_w / (p.visc_w + p.visc_o)
    assert abs(s[np.argmin(lt)] - sstar) < 1e-3
    fw = frac_flow(s, p)
    assert fw[0] == 0.0 and fw[-1] == 1.0 and np.all(np.diff(fw) >= 0)


def test_basis_orthonormal_by_quadrature():
    """The cell basis is L2-orthonormal (4-point Gauss, independent rule)."""
    p = make_problem("small3d", n=(2, 2, 2), nc=(1, 1, 1))
    g = Grid(p)
    x, w = np.polynomial.legendre.leggauss(4)
    P = np.array(np.meshgrid(x, x, x, indexing="ij")).reshape(3, -1).T
    W = np.prod(np.array(np.meshgrid(w, w, w, indexing="ij")).reshape(3, -1), axis=0) * g.vol / 8
    B = g.basis_at(P)
    assert np.allclose(B.T @ (W[:, None] * B), np.eye(4), atol=1e-13)


def _randomize_bcs(p, rng):
    bm = p.bc_type > 0
    p.bc_type[bm] = rng.choice([1, 2], bm.sum()).astype(np.int8)
    p.bc_val[:] = rng.uniform(-1, 1, len(p.bc_val))
    p.perm[:] = 1e-13 * np.exp(rng.normal(0, 1.5, p.ncell))
    p.q1[:] = rng.uniform(0, 1e-3, p.ncell)


@pytest.mark.parametrize("case", [("tiny2d", (2, 2, 1)), ("tiny2d", (3, 2, 1)), ("small3d", (2, 2, 2))])
@pytest.mark.parametrize("weights", [0, 1])
def test_brute_force_assembly(case, weights):
    """Vectorized SWIP assembly equals a naive per-element/per-face
    4-point-Gauss evaluation on tiny grids (random kappa, s, BCs)."""
    name, n = case
    p = make_problem(name, n=n, nc=(1, 1, 1))
    rng = np.random.default_rng(3)
    _randomize_bcs(p, rng)
    p.weights = weights
    g = Grid(p)
    s = random_saturation(p, rng)
    gam = Mobility(g, p, s=s)
    A = assemble(g, p, gam).toarray()
    l = rhs(g, p, gam)
    Ab, lb = brute_assemble(p, s)
    assert np.abs(A - Ab).max() <= 1e-13 * np.abs(Ab).max()
    assert np.abs(l - lb).max() <= 1e-13 * np.abs(lb).max()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    if weights == 0:
        # SWIP weights are bounded by the harmonic-mean penalty, so b_h stays
        # coercive at any contrast; the literal weights need not be
        assert np.linalg.eigvalsh(A).min() > 0


def _slab(dim, variant, kappa=None):
    """Box with Dirichlet p on x=0, Dirichlet or Neumann on x=L, no flow elsewhere."""
    p = make_problem("tiny2d" if dim == 2 else "small3d")
    g = Grid(p)
    p.q1[:] = 0
    p.q2[:] = 0
    p.perm[:] = 2e-13 if kappa is None else kappa
    p.bc_type[:] = 0
    p.bc_val[:] = 0
    for a in range(dim):
        fa = g.faces[a]
        p.bc_type[fa["gid"][(fa["lo"] < 0) | (fa["hi"] < 0)]] = 1
    f = g.faces[0]
    left, right = f["gid"][f["lo"] < 0], f["gid"][f["hi"] < 0]
    p.bc_type[left] = 2
    return p, g, left, right


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("variant", ["dirichlet", "neumann"])
def test_affine_pressure_reproduced(dim, variant):
    """SWIP is consistent: the affine solution p = beta x with constant
    lambda kappa lies in V_h and is reproduced exactly, with Dirichlet data
    on both ends or Dirichlet + the outward Neumann flux -lambda kappa beta.
    A '+' consistency sign or a '+ v_N' Neumann term fails this."""
    p, g, left, right = _slab(dim, variant)
    beta = 1e5
    s = np.zeros(g.r * g.ncell)
    s[:g.ncell] = 0.3 * math.sqrt(g.vol)
    lam = mobilities(np.array([0.3]), p)[2][0]
    p.bc_val[left] = 0.0
    if variant == "dirichlet":
        p.bc_type[right] = 2
        p.bc_val[right] = beta * g.L[0]
    else:
        p.bc_type[right] = 1
        p.bc_val[right] = -lam * 2e-13 * beta
    ph = fine_pressure(g, p, s=s)
    nc = g.ncell
    ex = np.zeros_like(ph)
    ex[:nc] = beta * g.centers[:, 0] * math.sqrt(g.vol)
    ex[nc:2 * nc] = beta * g.h[0] * math.sqrt(g.vol) / (2 * math.sqrt(3))
    assert np.abs(ph - ex).max() <= 1e-11 * np.abs(ex).max()
    F = reconstruct_flux(g, p, ph, Mobility(g, p, s=s))
    fx = F[g.faces[0]["gid"]]
    assert np.allclose(fx, -lam * 2e-13 * beta * g.faces[0]["area"], rtol=1e-9)


def test_layered_piecewise_linear_exact():
    """Piecewise-constant kappa in x-layers aligned with faces: the exact
    solution of the 1D flux problem is continuous piecewise linear (in V_h)
    and SWIP reproduces it exactly, with either mean weights."""
    p, g, left, right = _slab(2, "dirichlet")
    xi = g.ijk[:, 0]
    kap = np.where(xi < 3, 1e-13, np.where(xi < 6, 5e-12, 3e-14))
    p.perm[:] = kap
    p.bc_type[right] = 2
    p.bc_val[left], p.bc_val[right] = 1e6, 0.0
    s = np.zeros(g.r * g.ncell)          # lambda = 1/eta_o everywhere
    lam = 1.0 / p.visc_o
    # exact: flux q = (p_L - p_R) / sum_i (h / (lam kappa_i)) along x
    kx = np.array([1e-13] * 3 + [5e-12] * 3 + [3e-14] * 2)
    res = g.h[0] / (lam * kx)
    q = 1e6 / res.sum()
    pf = 1e6 - np.concatenate([[0.0], np.cumsum(q * res)])           # face values
    for weights in (0, 1):
        p.weights = weights
        ph = fine_pressure(g, p, s=s)
        nc = g.ncell
        i = g.ijk[:, 0]
        mean = 0.5 * (pf[i] + pf[i + 1])
        slope = 0.5 * (pf[i + 1] - pf[i])
        assert np.abs(ph[:nc] / math.sqrt(g.vol) - mean).max() <= 1e-10 * 1e6
        assert np.abs(ph[nc:2 * nc] * math.sqrt(3) / math.sqrt(g.vol) - slope).max() <= 1e-10 * 1e6


def _mms_error(n):
    p = make_problem("tiny2d", n=(n, n, 1), nc=(1, 1, 1))
    g = Grid(p)
    p.perm[:] = 1e-12
    p.q1[:] = 0
    p.bc_type[p.bc_type > 0] = 2
    p.bc_val[:] = 0.0
    s = np.zeros(g.r * g.ncell)
    s[:g.ncell] = math.sqrt(g.vol)       # s = 1: lambda = 1/eta_w, the largest mobility
    lam = 1.0 / p.visc_w
    A = assemble(g, p, Mobility(g, p, s=s))
    # l_k = int_e f phi_k, f = 2 pi^2 lam kappa sin(pi x) sin(pi y), 5-point Gauss
    x, w = np.polynomial.legendre.leggauss(5)
    XI = np.array(np.meshgrid(x, x, indexing="ij")).reshape(2, -1).T
    W = np.outer(w, w).ravel() * g.vol / 4
    B = g.basis_at(XI)
    pts = g.centers[:, None, :2] + 0.5 * XI[None] * g.h[None, None, :2]
    exact = np.sin(np.pi * pts[..., 0]) * np.sin(np.pi * pts[..., 1])
    f = 2 * np.pi ** 2 * lam * 1e-12 * exact
    l = np.concatenate([(f * W) @ B[:, k] for k in range(3)])
    ph = solve_spd(A, l)
    vals = np.stack([ph[k * g.ncell:(k + 1) * g.ncell] for k in range(3)], 1) @ B.T
    return math.sqrt(((vals - exact) ** 2 * W).sum())


def test_mms_second_order():
    """Smooth manufactured solution: L2 error of P1 SWIP falls like h^2."""
    e1, e2 = _mms_error(16), _mms_error(32)
    rate = math.log2(e1 / e2)
    assert 1.8 < rate < 2.3


def test_fine_flux_conservative():
    """Def. velocityDG with v_N on Neumann faces: every cell's net outward
    flux equals int_e q1 (to round-off) for the fine solution."""
    p = make_problem("small2d")
    g = Grid(p)
    s = random_saturation(p, np.random.default_rng(0))
    ph = fine_pressure(g, p, s=s)
    F = reconstruct_flux(g, p, ph, Mobility(g, p, s=s))
    out = cell_outflow(g, F)
    assert np.abs(out - p.q1 * g.vol).max() <= 1e-10 * np.abs(F).max()
