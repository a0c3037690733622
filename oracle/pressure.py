"""SWIP pressure discretization, fine solve and velocity reconstruction
(oracle; test infrastructure).

Follows Sec. 3.2 (eq. swipBilP, eq. penaltyParam and the Remark after it, the
linear form l_h, Def. pressureDG) and Sec. 3.3 (Def. velocityDG) with these
readings of the printed formulas:

* the consistency terms of b_h carry a minus sign (standard SWIP; the printed
  "+" contradicts the printed l_h Dirichlet term and the velocity formula);
* the Neumann term of l_h is -int v_N w, because the boundary condition
  defines v_N as the outward flux -lambda kappa grad p . n;
* the weighted mean uses the SWIP weights om1 = a2/(a1+a2) (option: the
  literal om_l = a_l/(a1+a2));
* on a Dirichlet face the one-sided trace has weight 1, sigma_f = c a1,
  the normal is the outward normal and [v] = v;
* h_f is the face diameter (face length in 2D, face diagonal in 3D);
* gravity is zero (the configurations have G = 0), so the gravity terms of
  l_h vanish;
* the mobility gamma may be two-valued on a face (it is lambda(s_h) with a
  discontinuous s_h): each side of the weighted mean uses its own trace.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import Grid, mobilities, penalty_sigma, mean_weights

BC_NEUMANN, BC_DIRICHLET = 1, 2


class Mobility:
    """Values of a mobility gamma at the 2-point Gauss points of cells and of
    cell faces.  Built either from a saturation (gamma = lambda(s)) or from a
    given P1 field (e.g. a mobility profile or a fitted combination)."""

    def __init__(self, grid: Grid, prob, s=None, field=None, phase="total"):
        assert (s is None) != (field is None)
        self.grid, self.prob, self.s, self.field, self.phase = grid, prob, s, field, phase

    def _apply(self, vals):
        if self.field is not None:
            return vals
        lw, lo, lt = mobilities(vals, self.prob)
        return {"total": lt, "w": lw, "o": lo}[self.phase]

    def _u(self):
        return self.field if self.field is not None else self.s

    def cell(self, c):
        pts, _ = self.grid.cell_qpts()
        return self._apply(self.grid.eval_field(self._u(), c, pts))

    def face(self, c, a, xi_a):
        pts, _ = self.grid.face_qpts(a, xi_a)
        return self._apply(self.grid.eval_field(self._u(), c, pts))


def _dofs(grid, cells):
    """(nf, r) global dof numbers of the given cells (SoA numbering)."""
    return np.stack([k * grid.ncell + cells for k in range(grid.r)], axis=1)


def _scatter(rows, cols, vals, dof_r, dof_c, local):
    nf, m, n = local.shape
    rows.append(np.repeat(dof_r, n, axis=1).ravel())
    cols.append(np.tile(dof_c, (1, m)).ravel())
    vals.append(local.ravel())


def _boundary_kinds(grid, a):
    f = grid.faces[a]
    lo, hi = f["lo"], f["hi"]
    # (mask, interior cell, local xi_a of the face in that cell, outward normal sign)
    return [((lo >= 0) & (hi < 0), lo, +1.0, +1.0), ((lo < 0) & (hi >= 0), hi, -1.0, -1.0)]


def assemble(grid: Grid, prob, gam: Mobility | None, vol=True, cons=True, pen=True):
    """Matrix of b_h(., .; gamma) restricted to the requested terms:
    vol  = sum_e int_e gamma kappa grad v . grad w,
    cons = -sum_f int_f ({gamma kappa grad v . n}[w] + {gamma kappa grad w . n}[v]),
    pen  = sum_f sigma_f / h_f int_f [v][w],
    with f over interior and Dirichlet faces.  Returns a CSR matrix."""
    nc, r = grid.ncell, grid.r
    G = grid.grad_basis()                       # (r, d)
    kap = np.asarray(prob.perm, dtype=np.float64)
    rows, cols, vals = [], [], []
    allc = np.arange(nc)
    if vol and gam is not None:
        _, w = grid.cell_qpts()
        ig = gam.cell(allc) @ w                 # int_e gamma
        K = G @ G.T
        local = (kap * ig)[:, None, None] * K[None]
        d = _dofs(grid, allc)
        _scatter(rows, cols, vals, d, d, local)
    for a in range(grid.dim):
        f = grid.faces[a]
        hf = f["hf"]
        m = (f["lo"] >= 0) & (f["hi"] >= 0)
        c0, c1 = f["lo"][m], f["hi"][m]
        p0, w = grid.face_qpts(a, +1.0)
        p1, _ = grid.face_qpts(a, -1.0)
        T0, T1 = grid.basis_at(p0), grid.basis_at(p1)      # (nq, r)
        J = [T0, -T1]                                       # jump contributions
        dn = G[:, a]                                        # d/dn with n = +e_a
        k0, k1 = kap[c0], kap[c1]
        dofs = np.concatenate([_dofs(grid, c0), _dofs(grid, c1)], axis=1)
        if cons and gam is not None:
            om0, om1 = mean_weights(prob, k0, k1)
            g0, g1 = gam.face(c0, a, +1.0), gam.face(c1, a, -1.0)
            blocks = []
            for oms, ks, gs in ((om0, k0, g0), (om1, k1, g1)):
                mom = np.concatenate([(gs * w) @ J[sp_] for sp_ in (0, 1)], axis=1)  # (nf, 2r)
                row = (oms * ks)[:, None] * dn[None, :]                           # (nf, r)
                blocks.append(row[:, :, None] * mom[:, None, :])                  # (nf, r, 2r)
            C = np.concatenate(blocks, axis=1)                                    # (nf, 2r, 2r)
            _scatter(rows, cols, vals, dofs, dofs, -(C + C.transpose(0, 2, 1)))
        if pen:
            sig = penalty_sigma(prob, k0, k1) / hf
            Jm = np.concatenate(J, axis=1)                                        # (nq, 2r)
            P = Jm.T @ (w[:, None] * Jm)
            _scatter(rows, cols, vals, dofs, dofs, sig[:, None, None] * P[None])
        for mask, cell, xi, nsgn in _boundary_kinds(grid, a):
            gid = f["gid"][mask]
            dm = prob.bc_type[gid] == BC_DIRICHLET
            cb = cell[mask][dm]
            if len(cb) == 0:
                continue
            pts, w = grid.face_qpts(a, xi)
            T = grid.basis_at(pts)
            dno = nsgn * G[:, a]
            kb = kap[cb]
            db = _dofs(grid, cb)
            if cons and gam is not None:
                gb = gam.face(cb, a, xi)
                mom = (gb * w) @ T                                                # (nf, r)
                C = (kb[:, None] * dno[None, :])[:, :, None] * mom[:, None, :]
                _scatter(rows, cols, vals, db, db, -(C + C.transpose(0, 2, 1)))
            if pen:
                sig = penalty_sigma(prob, kb) / hf
                P = T.T @ (w[:, None] * T)
                _scatter(rows, cols, vals, db, db, sig[:, None, None] * P[None])
    n = nc * r
    if not rows:
        return sp.csr_matrix((n, n))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


def rhs(grid: Grid, prob, gam: Mobility | None, part="all"):
    """Linear form l_h(w) (gravity zero):
    int q1 w - sum_{Neumann} int v_N w + sum_{Dirichlet} int (sigma/h w - gamma kappa grad w . n) p_D.
    part = "const" (gamma-free terms), "gamma" (the gamma term), "all"."""
    nc, r = grid.ncell, grid.r
    G = grid.grad_basis()
    kap = np.asarray(prob.perm, dtype=np.float64)
    l = np.zeros(nc * r)
    if part in ("all", "const"):
        # int_e q1 phi_0 = q1 |e| |e|^{-1/2}
        l[:nc] += np.asarray(prob.q1) * np.sqrt(grid.vol)
    for a in range(grid.dim):
        f = grid.faces[a]
        hf = f["hf"]
        for mask, cell, xi, nsgn in _boundary_kinds(grid, a):
            gid = f["gid"][mask]
            cells = cell[mask]
            pts, w = grid.face_qpts(a, xi)
            T = grid.basis_at(pts)
            tw = w @ T                                               # int_f phi_k
            bt = prob.bc_type[gid]
            val = prob.bc_val[gid]
            nm = bt == BC_NEUMANN
            dm = bt == BC_DIRICHLET
            if part in ("all", "const"):
                for k in range(r):
                    np.add.at(l, k * nc + cells[nm], -val[nm] * tw[k])
                    sig = penalty_sigma(prob, kap[cells[dm]]) / hf
                    np.add.at(l, k * nc + cells[dm], sig * val[dm] * tw[k])
            if part in ("all", "gamma") and gam is not None and dm.any():
                cd = cells[dm]
                ig = gam.face(cd, a, xi) @ w                         # int_f gamma
                dno = nsgn * G[:, a]
                for k in range(r):
                    np.add.at(l, k * nc + cd, -val[dm] * kap[cd] * ig * dno[k])
    return l


def fine_operator(grid, prob, gam):
    """Full b_h(.,.;gamma) matrix and l_h vector."""
    return assemble(grid, prob, gam), rhs(grid, prob, gam)


def solve_spd(A, b, refine=2):
    """Sparse direct solve (SuperLU) with a few steps of iterative refinement."""
    lu = spla.splu(A.tocsc())
    x = lu.solve(b)
    for _ in range(refine):
        x = x + lu.solve(b - A @ x)
    return x


def fine_pressure(grid, prob, s=None, field=None):
    """Def. pressureDG: p_h with b_h(p_h, w; gamma) = l_h(w) for all w in V_h.
    gamma = lambda(s) (from a saturation) or a given P1 mobility field."""
    gam = Mobility(grid, prob, s=s, field=field)
    A, l = fine_operator(grid, prob, gam)
    return solve_spd(A, l)


def reconstruct_flux(grid, prob, p, gam: Mobility):
    """Def. velocityDG: the RT0 velocity is given by its face fluxes
    int_f u.n = int_f -n.{gamma kappa grad p} + sigma_f/h_f [p]* ds.
    Returns one flux per face, oriented along +axis.  On Neumann faces the
    flux is the prescribed outward flux v_N |f| (reading of the definition
    that makes the fine solution exactly conservative cell by cell)."""
    nc = grid.ncell
    G = grid.grad_basis()
    kap = np.asarray(prob.perm, dtype=np.float64)
    F = np.zeros(grid.nface)
    pc = lambda cells: np.stack([p[k * nc + cells] for k in range(grid.r)], axis=1)
    for a in range(grid.dim):
        f = grid.faces[a]
        hf = f["hf"]
        dn = G[:, a]
        m = (f["lo"] >= 0) & (f["hi"] >= 0)
        c0, c1 = f["lo"][m], f["hi"][m]
        p0, w = grid.face_qpts(a, +1.0)
        p1, _ = grid.face_qpts(a, -1.0)
        T0, T1 = grid.basis_at(p0), grid.basis_at(p1)
        k0, k1 = kap[c0], kap[c1]
        om0, om1 = mean_weights(prob, k0, k1)
        P0, P1 = pc(c0), pc(c1)
        g0 = gam.face(c0, a, +1.0) @ w
        g1 = gam.face(c1, a, -1.0) @ w
        jump = (P0 @ T0.T - P1 @ T1.T) @ w                      # int_f [p]
        sig = penalty_sigma(prob, k0, k1) / hf
        F[f["gid"][m]] = -(om0 * k0 * g0 * (P0 @ dn) + om1 * k1 * g1 * (P1 @ dn)) + sig * jump
        for mask, cell, xi, nsgn in _boundary_kinds(grid, a):
            gid = f["gid"][mask]
            cells = cell[mask]
            bt = prob.bc_type[gid]
            val = prob.bc_val[gid]
            out = np.zeros(len(gid))
            nm = bt == BC_NEUMANN
            out[nm] = val[nm] * f["area"]
            dm = bt == BC_DIRICHLET
            if dm.any():
                cd = cells[dm]
                pts, w = grid.face_qpts(a, xi)
                T = grid.basis_at(pts)
                Pd = pc(cd)
                g = gam.face(cd, a, xi) @ w
                sig = penalty_sigma(prob, kap[cd]) / hf
                out[dm] = (-kap[cd] * g * (Pd @ (nsgn * dn))
                           + sig * ((Pd @ T.T) @ w - val[dm] * f["area"]))
            F[gid] = nsgn * out
    return F


def cell_outflow(grid, F):
    """Net outward flux of every cell, sum over its faces of F_f^out."""
    out = np.zeros(grid.ncell)
    for a in range(grid.dim):
        f = grid.faces[a]
        Fa = F[f["gid"]]
        lo, hi = f["lo"], f["hi"]
        ml, mh = lo >= 0, hi >= 0
        np.add.at(out, lo[ml], Fa[ml])
        np.add.at(out, hi[mh], -Fa[mh])
    return out
