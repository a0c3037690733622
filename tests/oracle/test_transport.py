"""Pins of the oracle's saturation step, limiter and time-of-flight."""
import math

import numpy as np
import pytest

from synth import make_problem, random_saturation
from oracle.fem import Grid, frac_flow
from oracle.pressure import Mobility, fine_pressure, reconstruct_flux
from oracle.transport import euler_step, limit, shock_detector, saturation_step
from oracle.tof import time_of_flight, cell_means


def _flow(name, s, **kw):
    p = make_problem(name, **kw)
    g = Grid(p)
    ph = fine_pressure(g, p, s=s(g) if callable(s) else s)
    F = reconstruct_flux(g, p, ph, Mobility(g, p, s=s(g) if callable(s) else s))
    return p, g, F


def test_uniform_water_state_preserved():
    """s = 1 everywhere with water injection (q2 = q1) and a conservative
    velocity is a steady state of the scheme: every coefficient unchanged."""
    one = lambda g: np.concatenate([np.full(g.ncell, math.sqrt(g.vol)), np.zeros(g.dim * g.ncell)])
    for name in ("small2d", "small3d"):
        p, g, F = _flow(name, one)
        s = one(g)
        sb = euler_step(g, p, s, F)
        assert np.abs(sb - s).max() <= 1e-10 * math.sqrt(g.vol)


def test_mass_balance_closed_box():
    """Closed box (no-flow boundary) with an injector and a producer source:
    the total pore volume of water changes by exactly dt * int q2, whatever
    the state and the fluxes (interior face terms telescope)."""
    p = make_problem("small2d")
    g = Grid(p)
    p.bc_type[p.bc_type == 2] = 1
    p.bc_val[:] = 0.0
    q = np.zeros(g.ncell)
    q[0] = 1e-4
    q[-1] = -1e-4
    p.q1[:] = q
    rng = np.random.default_rng(4)
    p.q2[:] = rng.uniform(-1e-5, 1e-5, g.ncell)
    s = random_saturation(p, rng)
    # any pressure field gives fluxes; the no-flow Neumann faces carry zero flux
    ph = rng.standard_normal(g.r * g.ncell) * 1e5
    F = reconstruct_flux(g, p, ph, Mobility(g, p, s=s))
    sb = euler_step(g, p, s, F)
    mass = lambda u: (p.poro * cell_means(g, u) * g.vol).sum()
    assert mass(sb) - mass(s) == pytest.approx(p.dt * (p.q2 * g.vol).sum(), rel=1e-9, abs=1e-18)


def _bl_problem(nx, visc_ratio=5.0):
    p = make_problem("tiny2d", n=(nx, 1, 1), L=(1.0, 1.0 / nx, 1.0), nc=(1, 1, 1), ratio=visc_ratio)
    g = Grid(p)
    p.q1[:] = 0
    p.q2[:] = 0
    p.perm[:] = 1e-13
    p.bc_type[:] = 0
    p.bc_type[g.faces[1]["gid"]] = 1
    fx = g.faces[0]
    left = fx["gid"][fx["lo"] < 0]
    right = fx["gid"][fx["hi"] < 0]
    p.bc_type[left] = 2
    p.bc_sat[left] = 1
    p.bc_sval[left] = 1.0
    p.bc_type[right] = 1
    return p, g


def _welge(p, x, t, u):
    """Buckley-Leverett solution with the Welge tangent (textbook)."""
    ss = np.linspace(1e-6, 1, 200001)
    fw = frac_flow(ss, p)
    dfw = np.gradient(fw, ss)
    i = np.argmin(np.abs(fw / ss - dfw)[1000:]) + 1000
    s_front = ss[i]
    xf = u * t * fw[i] / (s_front * 0.2)
    sat = np.zeros_like(x)
    behind = x < xf
    # rarefaction: x = u t f'(s) / phi for s >= s_front
    sr = ss[i:]
    xr = u * t * dfw[i:] / 0.2
    sat[behind] = np.interp(x[behind], xr[::-1], sr[::-1])
    return sat


def _bl_error(nx):
    p, g = _bl_problem(nx)
    u = 2e-5
    F = np.zeros(g.nface)
    F[g.faces[0]["gid"]] = u * g.faces[0]["area"]
    dfmax = 3.0
    p.dt = 0.2 * 0.2 * g.h[0] / (u * dfmax)
    t_end = 0.5 * 0.2 * 1.0 / (u * 2.0)
    nsteps = int(round(t_end / p.dt))
    s = np.zeros(g.r * g.ncell)
    for _ in range(nsteps):
        s, _ = saturation_step(g, p, s, F)
    mean = cell_means(g, s)
    ex = _welge(p, g.centers[:, 0], nsteps * p.dt, u)
    return np.abs(mean - ex).mean(), s, g


def test_buckley_leverett_converges():
    """1D Buckley-Leverett displacement (Welge tangent construction): the
    L1 error of the DG + limiter scheme falls under refinement."""
    e1, s1, g1 = _bl_error(50)
    e2, s2, g2 = _bl_error(100)
    assert e2 < 0.75 * e1
    assert e2 < 0.05
    vals = g2.eval_field(s2, np.arange(g2.ncell), g2.vertices())
    assert vals.min() > -0.1 and vals.max() < 1.1


def test_limiter_properties():
    p, g = _bl_problem(40)
    rng = np.random.default_rng(8)
    s = random_saturation(p, rng, slope=0.4)
    s[g.ncell:] *= 3.0                        # push vertex values out of [0, 1]
    F = np.zeros(g.nface)
    F[g.faces[0]["gid"]] = 1e-5 * g.faces[0]["area"]
    out, flags = limit(g, p, s, F)
    nc = g.ncell
    assert np.array_equal(out[:nc], s[:nc])                          # means kept
    ratio = out[nc:2 * nc] / np.where(s[nc:2 * nc] == 0, 1, s[nc:2 * nc])
    assert np.all((ratio >= -1e-15) & (ratio <= 1 + 1e-15))          # m in [0, 1]
    assert np.array_equal(out[nc:][np.repeat(flags == 0, 2)], s[nc:][np.repeat(flags == 0, 2)])
    assert flags.sum() > 0


def test_limiter_leaves_smooth_data():
    """A globally linear state with values inside [0, 1] and no jumps is
    not flagged and is returned unchanged."""
    p, g = _bl_problem(40)
    p.bc_sat[:] = 0                       # no inflow Dirichlet value to jump against
    nc = g.ncell
    s = np.zeros(g.r * nc)
    x = g.centers[:, 0]
    s[:nc] = (0.2 + 0.5 * x) * math.sqrt(g.vol)
    s[nc:2 * nc] = 0.5 * g.h[0] / 2 * math.sqrt(g.vol) / math.sqrt(3)
    F = np.zeros(g.nface)
    F[g.faces[0]["gid"]] = 1e-5 * g.faces[0]["area"]
    assert np.abs(shock_detector(g, p, s, F)).max() < 1e-8
    out, flags = limit(g, p, s, F)
    assert flags.sum() == 0 and np.array_equal(out, s)


def test_tof_uniform_flow_exact():
    """1D uniform flow u: tau = phi x / u lies in V_h and the upwind DG
    time-of-flight reproduces it exactly."""
    p, g = _bl_problem(16)
    u = 3e-6
    F = np.zeros(g.nface)
    F[g.faces[0]["gid"]] = u * g.faces[0]["area"]
    tau = time_of_flight(g, p, F)
    nc = g.ncell
    assert np.allclose(cell_means(g, tau), 0.2 * g.centers[:, 0] / u, rtol=1e-10)
    slope = tau[nc:2 * nc] * math.sqrt(3) / math.sqrt(g.vol)          # half-cell increment
    assert np.allclose(slope, 0.2 * g.h[0] / (2 * u), rtol=1e-10)
