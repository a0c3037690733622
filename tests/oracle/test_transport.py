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


def _strip_state(g, means, drops):
    """P1 state on a strip of cells along x: cell means and the change of s
    across each cell in x (orthonormal basis: mean coefficient mean sqrt|e|,
    x coefficient (change / 2) sqrt|e| / sqrt(3), vertex values mean +- change / 2)."""
    nc = g.ncell
    s = np.zeros(g.r * nc)
    s[:nc] = np.asarray(means) * math.sqrt(g.vol)
    s[nc:2 * nc] = np.asarray(drops) / 2 * math.sqrt(g.vol) / math.sqrt(3)
    return s


def test_limiter_gradient_scales_by_hand():
    """Five cells in a row with no flow (no shock detector contribution), so
    a cell is flagged exactly when a vertex value leaves [0, 1].  The gradient
    scales follow the case table of the limiter (Sec. 3.5): with
    g_i = grad s . (b_i - b) and d_i the difference of the cell means,
      cell 0: mean -0.2, flat         -> flagged, nothing to scale
      cell 1: mean 0.03, change 0.08  -> |g| < |d| on both sides: m = 1
      cell 2: mean 0.5,  change 1.2   -> left  g = -1.2, d = -0.47: m = 0.47/1.2
                                         right g =  1.2, d =  0.1:  m = 0.1/1.2
      cell 3: mean 0.6,  flat         -> inside [0, 1]: not flagged
      cell 4: mean 0.9,  change -0.4  -> left  g = 0.4, d = -0.3: g d < 0, m = 0
    and the limited slope is min_i m_i times the slope; the means stay."""
    p, g = _bl_problem(5)
    means = [-0.2, 0.03, 0.5, 0.6, 0.9]
    drops = [0.0, 0.08, 1.2, 0.0, -0.4]
    s = _strip_state(g, means, drops)
    out, flags = limit(g, p, s, np.zeros(g.nface))
    nc = g.ncell
    assert flags.tolist() == [1, 1, 1, 0, 1]
    assert np.array_equal(out[:nc], s[:nc])
    want = np.array([0.0, 0.08, 1.2 * (0.1 / 1.2), 0.0, 0.0])
    got = out[nc:2 * nc] * 2 / math.sqrt(g.vol) * math.sqrt(3)
    assert np.allclose(got, want, rtol=1e-12, atol=1e-15)
    assert np.array_equal(out[2 * nc:], s[2 * nc:])


def test_shock_detector_by_hand():
    """Piecewise-constant means under a flow in +x: the upstream interface
    of cell i > 0 is its left face, of cell 0 the inflow boundary with s_D = 1,
    so S(e) = |jump| |f| / (0.08 d sqrt(h_e) |e|) with h_e = diam(e) (Sec. 3.5
    shock detector; reading: absolute value of the face integral).  All
    values lie in [0, 1], so the limiter flags exactly the cells with S > 1
    (cell 4's small jump gives S < 1)."""
    p, g = _bl_problem(5)
    means = [0.9, 0.7, 0.7, 0.2, 0.21]
    s = _strip_state(g, means, [0.0] * 5)
    F = np.zeros(g.nface)
    F[g.faces[0]["gid"]] = 1e-5 * g.faces[0]["area"]
    S = shock_detector(g, p, s, F)
    hx, hy = 1.0 / 5, 1.0 / 5
    diam, vol, face = math.hypot(hx, hy), hx * hy, hy
    up = [1.0] + means[:-1]
    want = [abs(u - m) * face / (0.08 * 2 * math.sqrt(diam) * vol) for u, m in zip(up, means)]
    assert np.allclose(S, want, rtol=1e-12, atol=1e-14)
    assert [w > 1 for w in want] == [True, True, False, True, False]
    _, flags = limit(g, p, s, F)
    assert flags.tolist() == [1, 1, 0, 1, 0]
    # the same state under the reverse flow: the upstream faces are the right ones
    S_rev = shock_detector(g, p, s, -F)
    down = means[1:] + [None]
    want_rev = [abs(dn - m) * face / (0.08 * 2 * math.sqrt(diam) * vol) if dn is not None else 0.0
                for dn, m in zip(down, means)]
    assert np.allclose(S_rev, want_rev, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("name,n,L,axis", [("tiny2d", (4, 6, 1), (1.0, 1.2, 1.0), 1),
                                           ("small3d", (3, 4, 5), (1.0, 1.0, 2.0), 2)])
def test_tof_uniform_flow_along_y_and_z_exact(name, n, L, axis):
    """Uniform flow v along y (2D) or z (3D), entering through the whole
    lower boundary: tau = phi x_axis / v lies in V_h, so the upwind DG time of
    flight reproduces it exactly, with no slope in the other directions (the
    x-only pin cannot see a mistake in the indexing of the other axes)."""
    p = make_problem(name, n=n, L=L, nc=(1, 1, 1))
    p.poro[:] = 0.2
    g = Grid(p)
    v = 2e-6
    F = np.zeros(g.nface)
    F[g.faces[axis]["gid"]] = v * g.faces[axis]["area"]
    tau = time_of_flight(g, p, F)
    nc = g.ncell
    assert np.allclose(cell_means(g, tau), 0.2 * g.centers[:, axis] / v, rtol=1e-12)
    slope = tau[(axis + 1) * nc:(axis + 2) * nc] * math.sqrt(3) / math.sqrt(g.vol)
    assert np.allclose(slope, 0.2 * g.h[axis] / (2 * v), rtol=1e-12)
    for a in range(g.dim):
        if a != axis:
            assert np.abs(tau[(a + 1) * nc:(a + 2) * nc]).max() <= 1e-12 * np.abs(tau).max()


def _tof_error_growing_flow(ny):
    """Flow along y with v(y) = v0 (1 + y) on the unit height (face fluxes
    v(y_f) |f|; the RT0 field is then exactly v).  The weak form of the time
    of flight is the conservative d(v tau)/dy = phi, so tau = phi y / (v0 (1 + y));
    returns the relative L2 error of the P1 solution at the cell quadrature
    points."""
    p = make_problem("tiny2d", n=(3, ny, 1), L=(0.6, 1.0, 1.0), nc=(1, 1, 1))
    p.poro[:] = 0.2
    g = Grid(p)
    v0 = 2e-6
    f = g.faces[1]
    yf = np.where(f["hi"] >= 0, g.centers[np.maximum(f["hi"], 0), 1] - g.h[1] / 2,
                  g.centers[np.maximum(f["lo"], 0), 1] + g.h[1] / 2)
    F = np.zeros(g.nface)
    F[f["gid"]] = v0 * (1 + yf) * f["area"]
    tau = time_of_flight(g, p, F)
    pts, w = g.cell_qpts()
    vals = g.eval_field(tau, np.arange(g.ncell), pts)
    y = g.centers[:, 1][:, None] + pts[None, :, 1] * g.h[1] / 2
    exact = 0.2 * y / (v0 * (1 + y))
    return math.sqrt(((vals - exact) ** 2 @ w).sum() / (g.ncell * w.sum())) / (0.2 / v0)


def test_tof_growing_flow_second_order():
    """Non-uniform velocity (a source term in the flow): the P1 upwind DG
    time of flight converges at second order to the closed form."""
    e = [_tof_error_growing_flow(n) for n in (8, 16, 32)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(orders) >= 1.8, (e, orders)
    assert e[-1] < 1e-4


def test_saturation_penalty_by_hand():
    """No flow and no source: a piecewise-constant state changes only through
    the jump penalty of Def. saturationDG, - sum_f sigma_f / h_f int_f [s]* [v],
    on interior faces and on the saturation Dirichlet face (s_D = 1 on the
    left).  With sigma_f = scale (c_f / max eta) 2 k1 k2 / (k1 + k2) inside and
    scale (c_f / max eta) k on the boundary face (eq. penaltyParam; reading:
    h_f = face diameter), each cell mean moves by
    dt / (phi |e|) * sum over its faces of -sigma_f / h_f |f| (s_e - s_other)."""
    p, g = _bl_problem(3)
    p.q2[:] = 0.0
    p.poro[:] = 0.2
    p.perm[:] = [1e-13, 3e-13, 2e-13]
    p.sat_penalty_scale = 1.5
    means = [0.3, 0.8, 0.5]
    s = _strip_state(g, means, [0.0] * 3)
    c = 1.5 * p.penalty_c / max(p.visc_w, p.visc_o)
    k = [1e-13, 3e-13, 2e-13]
    h = 1.0 / 3                               # cell size, face length and face diameter
    area, vol = h, h * h
    sig01 = c * 2 * k[0] * k[1] / (k[0] + k[1])
    sig12 = c * 2 * k[1] * k[2] / (k[1] + k[2])
    sigb = c * k[0]
    dt = 0.05 * 0.2 * vol * h / (sig12 * area)     # moves of a few per cent
    flux = [-(sigb * (means[0] - 1.0) + sig01 * (means[0] - means[1])),
            -(sig01 * (means[1] - means[0]) + sig12 * (means[1] - means[2])),
            -(sig12 * (means[2] - means[1]))]
    want = [m + dt / (0.2 * vol) * f * area / h for m, f in zip(means, flux)]
    out = euler_step(g, p, s, np.zeros(g.nface), dt=dt)
    got = out[:g.ncell] / math.sqrt(vol)
    assert np.allclose(got - means, np.array(want) - means, rtol=1e-10, atol=0)
    assert abs(got[0] - means[0]) > 1e-3         # the moves are not negligible


def _dg1d_tof(v_faces, h, phi):
    """Textbook 1D P1 upwind DG for d(v tau)/dy = phi, v > 0 linear in each
    cell (face values v_faces), tau = 0 at the inflow: per cell tau = t0 + t1 xi
    (xi in [-1, 1]); testing with 1 and xi gives
      v_R (t0 + t1) - v_L T = phi h
      -(2 a t0 + 2/3 b t1) + v_R (t0 + t1) + v_L T = 0,
    a = (v_L + v_R)/2, b = (v_R - v_L)/2, T the upwind trace from below."""
    T, out = 0.0, []
    for vL, vR in zip(v_faces[:-1], v_faces[1:]):
        a, b = 0.5 * (vL + vR), 0.5 * (vR - vL)
        M = np.array([[vR, vR], [vR - 2 * a, vR - 2.0 / 3.0 * b]])
        t0, t1 = np.linalg.solve(M, [phi * h + vL * T, -vL * T])
        out.append((t0, t1))
        T = t0 + t1
    return np.array(out)


def test_tof_growing_flow_equals_1d_dg():
    """The same growing flow as above on a strip that is uniform in x: the
    oracle's DG time of flight equals, cell by cell, an independent 1D P1
    upwind DG solution (a change of the discrete scheme, even one of higher
    order such as the velocity interpolated along the wrong axis, shows here)."""
    ny, nx = 7, 3
    p = make_problem("tiny2d", n=(nx, ny, 1), L=(0.6, 1.0, 1.0), nc=(1, 1, 1))
    p.poro[:] = 0.2
    g = Grid(p)
    v0, h = 2e-6, 1.0 / ny
    f = g.faces[1]
    yf = np.where(f["hi"] >= 0, g.centers[np.maximum(f["hi"], 0), 1] - h / 2,
                  g.centers[np.maximum(f["lo"], 0), 1] + h / 2)
    F = np.zeros(g.nface)
    F[f["gid"]] = v0 * (1 + yf) * f["area"]
    tau = time_of_flight(g, p, F)
    ref = _dg1d_tof(v0 * (1 + np.arange(ny + 1) * h), h, 0.2)
    nc = g.ncell
    row = np.rint(g.centers[:, 1] / h - 0.5).astype(int)
    means = cell_means(g, tau)
    half = tau[2 * nc:3 * nc] * math.sqrt(3) / math.sqrt(g.vol)   # half-cell change in y
    assert np.allclose(means, ref[row, 0], rtol=1e-12)
    assert np.allclose(half, ref[row, 1], rtol=1e-10)
    assert np.abs(tau[nc:2 * nc]).max() <= 1e-12 * np.abs(tau).max()
