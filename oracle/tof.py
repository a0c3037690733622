"""DG time-of-flight (oracle; test infrastructure).

Eq. timeOfFlight (Sec. 3.6): find tau in V_h with, for every cell e and
psi in P1(e),
   -int_e tau u . grad psi + int_{de} tau^up (u . n_e) psi = int_e phi psi,
u the RT0 velocity of the face fluxes, tau^up the upwind trace (own trace
on outflow faces, neighbour trace on inflow faces, zero on inflow boundary
faces).  Solved here as one sparse linear system; the flow-ordered
block-triangular sweep is an equivalent way to solve the same system.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .transport import _cell_face_flux


def time_of_flight(grid, prob, F):
    nc, r, d = grid.ncell, grid.r, grid.dim
    G = grid.grad_basis()
    rows, cols, vals = [], [], []

    def add(ri, ci, v):
        rows.append(ri)
        cols.append(ci)
        vals.append(v)

    allc = np.arange(nc)
    pts, w = grid.cell_qpts()
    B = grid.basis_at(pts)                       # (nq, r)
    for a in range(d):
        Flo, Fhi = _cell_face_flux(grid, F, a)
        area = grid.faces[a]["area"]
        t = 0.5 * (1.0 + pts[:, a])
        ua = ((1.0 - t)[None, :] * Flo[:, None] + t[None, :] * Fhi[:, None]) / area  # (nc, nq)
        for k in range(r):
            # -int tau u_a d_a psi with psi = phi_{a+1}; tau = sum_k tau_k phi_k
            coef = -G[a + 1, a] * ((ua * w[None, :]) @ B[:, k])
            add((a + 1) * nc + allc, k * nc + allc, coef)
    for a in range(d):
        f = grid.faces[a]
        area = f["area"]
        Fa = F[f["gid"]]
        m = (f["lo"] >= 0) & (f["hi"] >= 0)
        c0, c1, Fi = f["lo"][m], f["hi"][m], Fa[m]
        p0, wf = grid.face_qpts(a, +1.0)
        p1, _ = grid.face_qpts(a, -1.0)
        T0, T1 = grid.basis_at(p0), grid.basis_at(p1)
        up0 = Fi >= 0.0
        # upwind cell and its trace basis per face
        for kt in range(r):
            for k in range(r):
                # test on c0 (outward flux +F), test on c1 (outward flux -F)
                m00 = (wf * T0[:, k] * T0[:, kt]).sum()
                m10 = (wf * T1[:, k] * T0[:, kt]).sum()
                m01 = (wf * T0[:, k] * T1[:, kt]).sum()
                m11 = (wf * T1[:, k] * T1[:, kt]).sum()
                # row c0
                add(kt * nc + c0[up0], k * nc + c0[up0], (Fi[up0] / area) * m00)
                add(kt * nc + c0[~up0], k * nc + c1[~up0], (Fi[~up0] / area) * m10)
                # row c1
                add(kt * nc + c1[up0], k * nc + c0[up0], (-Fi[up0] / area) * m01)
                add(kt * nc + c1[~up0], k * nc + c1[~up0], (-Fi[~up0] / area) * m11)
        for xi, nsgn, cellarr, mask in ((+1.0, +1.0, f["lo"], (f["lo"] >= 0) & (f["hi"] < 0)),
                                        (-1.0, -1.0, f["hi"], (f["lo"] < 0) & (f["hi"] >= 0))):
            cb = cellarr[mask]
            fout = nsgn * F[f["gid"][mask]]
            out = fout >= 0.0
            pts_b, wb = grid.face_qpts(a, xi)
            T = grid.basis_at(pts_b)
            for kt in range(r):
                for k in range(r):
                    mm = (wb * T[:, k] * T[:, kt]).sum()
                    add(kt * nc + cb[out], k * nc + cb[out], (fout[out] / area) * mm)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(r * nc, r * nc)).tocsc()
    b = np.zeros(r * nc)
    b[:nc] = np.asarray(prob.poro) * math.sqrt(grid.vol)
    return spla.splu(A).solve(b)


def cell_means(grid, u):
    return u[:grid.ncell] / math.sqrt(grid.vol)
