"""DG upwind explicit Euler saturation step and slope limiter (oracle; test
infrastructure).

Def. saturationDG (Sec. 3.4), with gravity zero:
  int_e phi/dt s^{n+1} v = int_e phi/dt s^n v + int_e q2 v
                          + int_e u f_w(s^n) . grad v
                          - sum_f int_f (u.n) f_w(chi(s^n)) [v]
                          - sum_{f in interior + Gamma_sd} sigma_f/h_f int_f [s^n]* [v]
Readings: u is the rectangular RT0 field of the face fluxes (u_a linear in
x_a only); chi is the upwind trace on interior faces (flux >= 0 takes the
low-side cell, as printed), s_D on saturation Dirichlet faces and the interior
trace on the other boundary faces; [s]* = s - s_D on Gamma_sd; the source
term is int_e q2 v; sigma_f is the pressure penalty (eq. penaltyParam) times
an optional scale; integrals of f_w use the 2-point Gauss rules.

Limiter (Sec. 3.5, eq. limiterMain): shock detector over inflow faces (net
outward flux < 0) with |int_f [s]| per face, flag S > 1 or a vertex value
outside [0, 1]; gradient scales m_i against face neighbours; the limited
state keeps the cell mean and scales the slope by min_i m_i.
"""
from __future__ import annotations

import math

import numpy as np

from .fem import frac_flow, penalty_sigma


def _cell_face_flux(grid, F, a):
    """Fluxes (along +axis) through the low and high face of every cell."""
    f = grid.faces[a]
    Flo = np.zeros(grid.ncell)
    Fhi = np.zeros(grid.ncell)
    Fa = F[f["gid"]]
    mh = f["hi"] >= 0
    Flo[f["hi"][mh]] = Fa[mh]          # the face is the low face of its hi cell
    ml = f["lo"] >= 0
    Fhi[f["lo"][ml]] = Fa[ml]
    return Flo, Fhi


def euler_step(grid, prob, s, F, dt=None):
    """Returns the unlimited state s-bar^{n+1} (SoA coefficients)."""
    dt = prob.dt if dt is None else dt
    nc, r, d = grid.ncell, grid.r, grid.dim
    G = grid.grad_basis()
    kap = np.asarray(prob.perm, dtype=np.float64)
    R = np.zeros(r * nc)
    allc = np.arange(nc)
    R[:nc] += np.asarray(prob.q2) * math.sqrt(grid.vol)
    pts, w = grid.cell_qpts()
    fw = frac_flow(grid.eval_field(s, allc, pts), prob)           # (nc, nq)
    for a in range(d):
        Flo, Fhi = _cell_face_flux(grid, F, a)
        area = grid.faces[a]["area"]
        t = 0.5 * (1.0 + pts[:, a])
        ua = ((1.0 - t)[None, :] * Flo[:, None] + t[None, :] * Fhi[:, None]) / area
        R[(a + 1) * nc:(a + 2) * nc] += G[a + 1, a] * ((ua * fw) @ w)
    sps = prob.sat_penalty_scale
    for a in range(d):
        f = grid.faces[a]
        hf, area = f["hf"], f["area"]
        Fa = F[f["gid"]]
        m = (f["lo"] >= 0) & (f["hi"] >= 0)
        c0, c1, Fi = f["lo"][m], f["hi"][m], Fa[m]
        p0, wf = grid.face_qpts(a, +1.0)
        p1, _ = grid.face_qpts(a, -1.0)
        T0, T1 = grid.basis_at(p0), grid.basis_at(p1)
        s0 = grid.eval_field(s, c0, p0)
        s1 = grid.eval_field(s, c1, p1)
        sup = np.where((Fi >= 0.0)[:, None], s0, s1)
        g = (Fi / area)[:, None] * frac_flow(sup, prob)                # (nf, nq)
        sig = sps * penalty_sigma(prob, kap[c0], kap[c1]) / hf
        jmp = sig[:, None] * (s0 - s1)
        tot = g + jmp
        for k in range(r):
            np.add.at(R, k * nc + c0, -(tot * wf) @ T0[:, k])
            np.add.at(R, k * nc + c1, (tot * wf) @ T1[:, k])
        for xi, nsgn, cellarr, mask in ((+1.0, +1.0, f["lo"], (f["lo"] >= 0) & (f["hi"] < 0)),
                                        (-1.0, -1.0, f["hi"], (f["lo"] < 0) & (f["hi"] >= 0))):
            cb = cellarr[mask]
            gid = f["gid"][mask]
            if len(cb) == 0:
                continue
            pts_b, wb = grid.face_qpts(a, xi)
            T = grid.basis_at(pts_b)
            sb = grid.eval_field(s, cb, pts_b)
            fout = nsgn * F[gid]
            sd = prob.bc_sat[gid] == 1
            sval = prob.bc_sval[gid]
            chi = np.where(sd[:, None], sval[:, None], sb)
            g = (fout / area)[:, None] * frac_flow(chi, prob)
            sig = sps * penalty_sigma(prob, kap[cb]) / hf
            jmp = np.where(sd[:, None], sig[:, None] * (sb - sval[:, None]), 0.0)
            tot = g + jmp
            for k in range(r):
                np.add.at(R, k * nc + cb, -(tot * wb) @ T[:, k])
    phi = np.asarray(prob.poro, dtype=np.float64)
    return s + dt * R / np.tile(phi, r)


def _mcase(g, dlt):
    """Gradient scale m_i of the limiter for neighbour differences g_i, d_i."""
    big = (np.abs(g) > 1e-8) & (np.abs(dlt) > 1e-8)
    m = np.ones_like(g)
    m = np.where(big & (g * dlt < 0), 0.0, m)
    sel = big & (g * dlt > 0) & (np.abs(g) > np.abs(dlt))
    m = np.where(sel, dlt / np.where(sel, g, 1.0), m)
    return m


def shock_detector(grid, prob, s, F):
    """S(e) = sum over inflow faces of |int_f [s]*| / (0.08 d sqrt(h_e) |e|)."""
    nc, d = grid.ncell, grid.dim
    S = np.zeros(nc)
    for a in range(d):
        f = grid.faces[a]
        Fa = F[f["gid"]]
        m = (f["lo"] >= 0) & (f["hi"] >= 0)
        c0, c1, Fi = f["lo"][m], f["hi"][m], Fa[m]
        p0, wf = grid.face_qpts(a, +1.0)
        p1, _ = grid.face_qpts(a, -1.0)
        J = np.abs((grid.eval_field(s, c0, p0) - grid.eval_field(s, c1, p1)) @ wf)
        np.add.at(S, c0[Fi < 0], J[Fi < 0])        # outward flux of c0 is +F
        np.add.at(S, c1[Fi > 0], J[Fi > 0])        # outward flux of c1 is -F
        for xi, nsgn, cellarr, mask in ((+1.0, +1.0, f["lo"], (f["lo"] >= 0) & (f["hi"] < 0)),
                                        (-1.0, -1.0, f["hi"], (f["lo"] < 0) & (f["hi"] >= 0))):
            gid = f["gid"][mask]
            cb = cellarr[mask]
            sd = prob.bc_sat[gid] == 1
            inflow = (nsgn * F[gid] < 0) & sd
            if inflow.any():
                pts, wb = grid.face_qpts(a, xi)
                J = np.abs((grid.eval_field(s, cb[inflow], pts) - prob.bc_sval[gid][inflow][:, None]) @ wb)
                np.add.at(S, cb[inflow], J)
    return S / (0.08 * d * math.sqrt(grid.he) * grid.vol)


def limit(grid, prob, s, F):
    """Slope limiter.  Returns (limited state, uint8 flags)."""
    nc, d = grid.ncell, grid.dim
    sq = math.sqrt(grid.vol)
    mean = s[:nc] / sq
    vals = grid.eval_field(s, np.arange(nc), grid.vertices())
    outside = ((vals < 0.0) | (vals > 1.0)).any(axis=1)
    S = shock_detector(grid, prob, s, F)
    flag = (S > 1.0) | outside
    G = grid.grad_basis()
    mmin = np.ones(nc)
    for a in range(d):
        f = grid.faces[a]
        m = (f["lo"] >= 0) & (f["hi"] >= 0)
        c0, c1 = f["lo"][m], f["hi"][m]
        ga = lambda c: G[a + 1, a] * s[(a + 1) * nc + c]        # d s / d x_a
        h = grid.h[a]
        m0 = _mcase(ga(c0) * h, mean[c1] - mean[c0])
        m1 = _mcase(ga(c1) * (-h), mean[c0] - mean[c1])
        np.minimum.at(mmin, c0, m0)
        np.minimum.at(mmin, c1, m1)
    out = s.copy()
    scale = np.where(flag, mmin, 1.0)
    for a in range(d):
        out[(a + 1) * nc:(a + 2) * nc] *= scale
    return out, flag.astype(np.uint8)


def saturation_step(grid, prob, s, F, dt=None):
    """One step: Euler update, then the limiter when enabled."""
    sb = euler_step(grid, prob, s, F, dt)
    if prob.limiter:
        return limit(grid, prob, sb, F)
    return sb, np.zeros(grid.ncell, dtype=np.uint8)
