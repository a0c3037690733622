"""Offline stage of the LRBMS method (oracle; test infrastructure).

Sec. 4.3 Alg. 2 (LRBMS basis construction) and Sec. 4.4 (offline-online
decomposition):
  * initial pressure/velocity and time-of-flight (Alg. 2 step 1a-1b);
  * mobility profiles from the time-of-flight (Alg. 2 step 1c), tested on the
    cell mean of tau so that every profile lies in V_h; T = the simulated
    horizon (the problem's t_end, else N_T dt);
  * snapshots at training mobilities gamma = sum_q mu_q Lambda^q;
  * local bases per coarse box E: optional unit function 1_E first, then
    Gram-Schmidt in L2(E) with rejection of relative norms <= 1e-8
    (Alg. 2 step 2e), or PCA by the method of snapshots with discarded
    energy <= eps^2 of the total (Alg. 2 step 3); a cap on N_E;
  * the greedy loop with the true energy-norm error (Alg. 2 step 2 with the
    error measure of Sec. 6) over a training set;
  * the affine terms b_q, c, d_q, e (Sec. 4.4).
Coarse boxes are numbered lexicographically (x fastest); within a box cells
are listed x fastest.  A local basis function is stored as an (r, n_E) array
of cell coefficients.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .fem import mobilities
from .pressure import Mobility, assemble, rhs, fine_pressure, reconstruct_flux
from .tof import time_of_flight, cell_means


def subdomain_cells(grid, prob):
    """Cell lists of the coarse boxes (lexicographic boxes, x-fastest cells)."""
    cuts = [np.asarray(c) for c in prob.cuts]
    boxes = []
    nx, ny, _ = grid.n
    for ez in range(len(cuts[2]) - 1):
        for ey in range(len(cuts[1]) - 1):
            for ex in range(len(cuts[0]) - 1):
                kk, jj, ii = np.meshgrid(np.arange(cuts[2][ez], cuts[2][ez + 1]),
                                         np.arange(cuts[1][ey], cuts[1][ey + 1]),
                                         np.arange(cuts[0][ex], cuts[0][ex + 1]), indexing="ij")
                boxes.append((ii + nx * (jj + ny * kk)).ravel())
    return boxes


def restrict(grid, u, cells):
    return np.stack([u[k * grid.ncell + cells] for k in range(grid.r)], axis=0)


def unit_function(grid, cells):
    """1_E normalized in L2(E): only the mean coefficient, |e|^{1/2}/|E|^{1/2}."""
    v = np.zeros((grid.r, len(cells)))
    v[0, :] = math.sqrt(grid.vol)
    return v / np.linalg.norm(v)


def gs_extend(basis, v, tol=1e-8):
    """Two-pass Gram-Schmidt of v against basis (L2(E) = coefficient dot
    product); appends v/|v| unless the remaining norm is <= tol * |v|."""
    nv = np.linalg.norm(v)
    if nv == 0.0:
        return False
    w = v.copy()
    for _ in range(2):
        for b in basis:
            w = w - np.vdot(b, w) * b
    nw = np.linalg.norm(w)
    if nw <= tol * nv:
        return False
    basis.append(w / nw)
    return True


def pca_modes(vecs, eps):
    """Method of snapshots: fewest modes whose discarded energy is <= eps^2 of
    the total energy."""
    if not vecs:
        return []
    X = np.stack([v.ravel() for v in vecs], axis=1)               # (L, ns)
    C = X.T @ X
    lam, V = np.linalg.eigh(C)
    order = np.argsort(lam)[::-1]
    lam, V = lam[order], V[:, order]
    lam = np.maximum(lam, 0.0)
    tot = lam.sum()
    if tot <= 0:
        return []
    keep = len(lam)
    for m in range(1, len(lam) + 1):
        if lam[m:].sum() <= eps ** 2 * tot:
            keep = m
            break
    modes = []
    for i in range(keep):
        if lam[i] <= 1e-30 * tot:
            break
        modes.append((X @ V[:, i] / math.sqrt(lam[i])).reshape(vecs[0].shape))
    return modes


def local_bases(grid, prob, snapshots, method=None, cap=None, unit=None, eps=None):
    """Local reduced bases Phi^E from global snapshots (list of SoA vectors)."""
    method = method or prob.basis_method
    cap = prob.ne_cap if cap is None else cap
    unit = prob.unit_functions if unit is None else unit
    eps = prob.pca_eps if eps is None else eps
    out = []
    for cells in subdomain_cells(grid, prob):
        basis = [unit_function(grid, cells)] if unit else []
        if method == "gs":
            for p in snapshots:
                if len(basis) >= cap:
                    break
                gs_extend(basis, restrict(grid, p, cells))
        elif method == "pca":
            vecs = []
            for p in snapshots:
                v = restrict(grid, p, cells)
                for b in basis:
                    v = v - np.vdot(b, v) * b
                vecs.append(v)
            for mode in pca_modes(vecs, eps):
                if len(basis) >= cap:
                    break
                gs_extend(basis, mode)
        elif method == "full":
            # every fine dof of E as its own basis function (T_H local spaces = V_h|E)
            basis = []
            for k in range(grid.r):
                for i in range(len(cells)):
                    v = np.zeros((grid.r, len(cells)))
                    v[k, i] = 1.0
                    basis.append(v)
        else:
            raise ValueError(method)
        out.append(np.stack(basis, axis=0))
    return out


class Basis:
    """Global reduced basis Phi_N = union of the local bases (Sec. 4.2)."""

    def __init__(self, grid, prob, phis):
        self.grid = grid
        self.cells = subdomain_cells(grid, prob)
        self.phis = [np.asarray(p, dtype=np.float64) for p in phis]
        self.sizes = np.array([p.shape[0] for p in self.phis], dtype=np.int64)
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self.N = int(self.offsets[-1])

    def matrix(self):
        """Sparse (r*ncell) x N matrix whose columns are the basis functions."""
        nc = self.grid.ncell
        rows, cols, vals = [], [], []
        for E, (cells, phi) in enumerate(zip(self.cells, self.phis)):
            NE, r, nE = phi.shape
            dof = (np.arange(r)[:, None] * nc + cells[None, :]).ravel()   # (r*nE)
            for j in range(NE):
                rows.append(dof)
                cols.append(np.full(r * nE, self.offsets[E] + j))
                vals.append(phi[j].ravel())
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(nc * self.grid.r, self.N))

    def flat(self):
        """Concatenation of the per-box arrays (N_E, r, n_E), C order."""
        return np.concatenate([p.ravel() for p in self.phis])


def mobility_profiles(grid, prob, tau, M, T):
    """Total-mobility profiles Lambda^1..Lambda^M (Alg. 2 step 1c) as P1
    fields (mean coefficient only).  Lambda^1 = lambda(0), Lambda^M =
    lambda(1), Lambda^q = lambda(0) where the cell-mean time-of-flight exceeds
    (q-1) T/(M-2), else lambda(1)."""
    nc = grid.ncell
    tb = cell_means(grid, tau)
    l0 = mobilities(np.array([0.0]), prob)[2][0]
    l1 = mobilities(np.array([1.0]), prob)[2][0]
    out = []
    for q in range(1, M + 1):
        if q == 1:
            val = np.full(nc, l0)
        elif q == M:
            val = np.full(nc, l1)
        else:
            val = np.where(tb > (q - 1) * T / (M - 2), l0, l1)
        fld = np.zeros(grid.r * nc)
        fld[:nc] = val * math.sqrt(grid.vol)
        out.append(fld)
    return out


def dedupe_profiles(profiles, rtol=1e-12):
    """Indices of a linearly independent subset (pivoted QR on the profile
    coefficient vectors; columns with |R_kk| < rtol * max are dropped)."""
    X = np.stack(profiles, axis=1)
    _, R, piv = sla.qr(X, mode="economic", pivoting=True)
    d = np.abs(np.diag(R))
    keep = piv[d > rtol * d.max()]
    return sorted(int(k) for k in keep)


def training_mobility(profiles, mu):
    return sum(m * p for m, p in zip(mu, profiles))


def initial_flow(grid, prob, s0=None):
    s0 = np.zeros(grid.r * grid.ncell) if s0 is None else s0
    p0 = fine_pressure(grid, prob, s=s0)
    F0 = reconstruct_flux(grid, prob, p0, Mobility(grid, prob, s=s0))
    return p0, F0


def build_offline(grid, prob, params, s0=None):
    """Alg. 2 without the greedy selection: profiles from the initial
    time-of-flight, one fine snapshot per training parameter (in order), local
    bases by Gram-Schmidt or PCA.  Returns a dict with everything."""
    p0, F0 = initial_flow(grid, prob, s0)
    tau = time_of_flight(grid, prob, F0)
    T = prob.t_end if prob.t_end > 0 else prob.n_steps * prob.dt
    profiles = mobility_profiles(grid, prob, tau, prob.M, T)
    snaps = [fine_pressure(grid, prob, field=training_mobility(profiles, mu)) for mu in params]
    phis = local_bases(grid, prob, snaps)
    keep = dedupe_profiles(profiles)
    return dict(p0=p0, F0=F0, tau=tau, profiles=profiles, keep=keep, snapshots=snaps,
                basis=Basis(grid, prob, phis))


def energy_error(grid, prob, A_bar, pH, ph):
    e = pH - ph
    return math.sqrt(max(float(e @ (A_bar @ e)), 0.0))


def greedy(grid, prob, profiles, params, n_max, tol, mu_bar=None):
    """Alg. 2 step 2 with the true error measure of Sec. 6: the fine
    snapshots of the whole training set are computed up front; in each
    iteration the worst-approximated parameter (energy norm of b_h(.,.;
    lambda-bar)) extends every local basis by Gram-Schmidt.  Stops when the
    maximum error is <= tol or the total size reaches n_max.  Returns
    (local bases, selected indices, max error history)."""
    mu_bar = np.full(len(profiles), 1.0 / len(profiles)) if mu_bar is None else mu_bar
    A_bar = assemble(grid, prob, Mobility(grid, prob, field=training_mobility(profiles, mu_bar)))
    fine = []
    ops = []
    for mu in params:
        gam = Mobility(grid, prob, field=training_mobility(profiles, mu))
        A = assemble(grid, prob, gam)
        l = rhs(grid, prob, gam)
        from .pressure import solve_spd
        fine.append(solve_spd(A, l))
        ops.append((A, l))
    cells = subdomain_cells(grid, prob)
    local = [[] for _ in cells]
    chosen, hist = [], []
    while True:
        errs = []
        total = sum(len(b) for b in local)
        for (A, l), ph in zip(ops, fine):
            if total == 0:
                pH = np.zeros_like(ph)
            else:
                B = Basis(grid, prob, [np.stack(b) if b else np.zeros((0, grid.r, len(c)))
                                       for b, c in zip(local, cells)]).matrix()
                An = (B.T @ (A @ B)).toarray()
                pH = B @ np.linalg.solve(An, B.T @ l)
            errs.append(energy_error(grid, prob, A_bar, pH, ph))
        k = int(np.argmax(errs))
        hist.append(errs[k])
        if errs[k] <= tol or total >= n_max:
            break
        chosen.append(k)
        grew = False
        for E, c in enumerate(cells):
            grew |= gs_extend(local[E], restrict(grid, fine[k], c))
        if not grew:
            break
    return [np.stack(b) if b else np.zeros((0, grid.r, len(c))) for b, c in zip(local, cells)], chosen, hist


def galerkin(B, A):
    """Phi^T A Phi: the reduced matrix of a fine operator A for the basis
    matrix B (columns = basis functions), accumulated in extended precision
    (x87 long double) and rounded once.  The reduced matrices of strongly
    heterogeneous problems are ill conditioned (2-norm condition ~1e9 at
    256 x 256, sigma_logk = 2) and their entries are sums with heavy
    cancellation (the penalty term pairs values on both sides of every fine
    face), so the rounding of a plain double evaluation moves the reduced
    solution by ~1e-10 on its own; rounded once, the entries carry only the
    rounding of the fine operator."""
    Bl = B.astype(np.longdouble)
    return (Bl.T @ (A.astype(np.longdouble) @ Bl)).tocsr().astype(np.float64)


def project(B, l):
    """Phi^T l, accumulated in extended precision and rounded once."""
    return np.asarray(B.T.astype(np.longdouble) @ np.asarray(l, dtype=np.longdouble),
                      dtype=np.float64)


def affine_terms(grid, prob, basis: Basis, profiles):
    """Sec. 4.4: c = Phi^T P Phi (penalty), b_q = Phi^T K(Lambda^q) Phi (volume
    and consistency terms), e = Phi^T l (gamma-free part), d_q = Phi^T l
    (gamma part with gamma = Lambda^q).  Sparse N x N matrices."""
    B = basis.matrix()
    P = assemble(grid, prob, None, vol=False, cons=False, pen=True)
    c = galerkin(B, P)
    e = project(B, rhs(grid, prob, None, part="const"))
    bq, dq = [], []
    for prof in profiles:
        gam = Mobility(grid, prob, field=prof)
        K = assemble(grid, prob, gam, vol=True, cons=True, pen=False)
        bq.append(galerkin(B, K))
        dq.append(project(B, rhs(grid, prob, gam, part="gamma")))
    return dict(c=c, e=e, b=bq, d=dq)
