"""Online stage of the LRBMS method (oracle; test infrastructure).

Alg. 3 step 5 for one time step:
  a) mobility of s^n; reduced system A_N p_N = f_N assembled
       AFFINE      c + sum_q theta_q b_q,  e + sum_q theta_q d_q
                   (eq. reducedSystem) with theta from the least-squares fit
                   (eq. leastSquaresFit) in L2 of the P1 projection of
                   lambda(s) (= l2 of orthonormal coefficients);
       DIRECT      Phi^T A(lambda(s^n)) Phi, Phi^T l(lambda(s^n)) (the
                   Galerkin projection of Def. coarseScalePressure with the
                   exact mobility, evaluated with the 2-point Gauss rules);
       DIRECT_FIT  the same with gamma = sum_q theta_q Lambda^q;
     and solved (dense Cholesky up to N = 2000, SuperLU above; iterative
     refinement with extended-precision residuals);
  b) p_h = sum_i (p_N)_i phi_i;
  c) face fluxes by Def. velocityDG with lambda(s^n) and p_h;
  d) saturation step (Def. saturationDG) and the limiter.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import Grid
from .pressure import Mobility, assemble, rhs, reconstruct_flux
from .transport import saturation_step
from .offline import Basis, affine_terms, galerkin, project, training_mobility

DIRECT, DIRECT_FIT, AFFINE = 0, 1, 2


def projected_mobility(grid, prob, s):
    """Coefficients of the L2 projection of lambda(s_h) onto V_h:
    int_e lambda(s) phi_k, 2-point Gauss."""
    nc = grid.ncell
    pts, w = grid.cell_qpts()
    lam = Mobility(grid, prob, s=s).cell(np.arange(nc))          # (nc, nq)
    B = grid.basis_at(pts)                                       # (nq, r)
    out = np.empty(grid.r * nc)
    for k in range(grid.r):
        out[k * nc:(k + 1) * nc] = (lam * w[None, :]) @ B[:, k]
    return out


def lsq_theta(grid, prob, s, profiles):
    """eq. leastSquaresFit: theta minimizing |Pi lambda(s) - sum theta_q Lambda^q|
    over linearly independent profiles (normal equations, Cholesky)."""
    X = np.stack(profiles, axis=1)
    r = X.T @ projected_mobility(grid, prob, s)
    Gm = X.T @ X
    return sla.cho_solve(sla.cho_factor(Gm), r)


class Model:
    """Reduced model: basis + (for AFFINE) profiles and affine terms."""

    def __init__(self, prob, phis, profiles=None):
        self.prob = prob
        self.grid = Grid(prob)
        self.basis = Basis(self.grid, prob, phis)
        self.B = self.basis.matrix()
        self.profiles = profiles
        self.terms = affine_terms(self.grid, prob, self.basis, profiles) if profiles else None


def assemble_direct(model: Model, gam: Mobility):
    A = assemble(model.grid, model.prob, gam)
    l = rhs(model.grid, model.prob, gam)
    B = model.B
    return galerkin(B, A), project(B, l)


def assemble_affine(model: Model, theta):
    """c + sum_q theta_q b_q and e + sum_q theta_q d_q (eq. reducedSystem),
    summed in extended precision and rounded once."""
    t = model.terms
    A = t["c"].astype(np.longdouble)
    f = np.asarray(t["e"], dtype=np.longdouble)
    for th, b, d in zip(theta, t["b"], t["d"]):
        A = A + np.longdouble(th) * b.astype(np.longdouble)
        f = f + np.longdouble(th) * np.asarray(d, dtype=np.longdouble)
    return A.tocsr().astype(np.float64), np.asarray(f, dtype=np.float64)


def reduced_system(model: Model, s, mode=DIRECT):
    g, p = model.grid, model.prob
    if mode == DIRECT:
        return assemble_direct(model, Mobility(g, p, s=s))
    theta = lsq_theta(g, p, s, model.profiles)
    if mode == AFFINE:
        return assemble_affine(model, theta)
    if mode == DIRECT_FIT:
        return assemble_direct(model, Mobility(g, p, field=training_mobility(model.profiles, theta)))
    raise ValueError(mode)


def solve_reduced(A, f, refine=3):
    """SPD solve with iterative refinement; residuals in extended precision."""
    n = A.shape[0]
    Al = A.astype(np.longdouble) if sp.issparse(A) else np.asarray(A, dtype=np.longdouble)
    fl = np.asarray(f, dtype=np.longdouble)
    if n <= 2000:
        Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
        fac = sla.cho_factor(Ad)
        sol = lambda b: sla.cho_solve(fac, b)
    else:
        lu = spla.splu(sp.csc_matrix(A))
        sol = lu.solve
    x = sol(np.asarray(f, dtype=np.float64))
    for _ in range(refine):
        res = fl - Al @ x.astype(np.longdouble)
        x = x + sol(np.asarray(res, dtype=np.float64))
    return x


def condition_estimate(A):
    """1-norm condition number estimate |A|_1 |A^-1|_1 of the reduced matrix
    (Hager/Higham estimator of |A^-1|_1 through LU solves), reported beside
    parity figures: two backward-stable solutions differ by about cond * eps."""
    A = sp.csc_matrix(A)
    lu = spla.splu(A)
    op = spla.LinearOperator(A.shape, matvec=lu.solve, rmatvec=lambda x: lu.solve(x, trans="T"),
                             dtype=np.float64)
    return float(spla.norm(A, 1) * spla.onenormest(op))


def reconstruct_pressure(model: Model, pN):
    """p_h^r = sum_i (p_N)_i phi_i (Alg. 3 step 5b)."""
    return model.B @ pN


def online_step(model: Model, s, mode=DIRECT, dt=None):
    """One online step.  Returns a dict with A_N, f_N, p_N, p_h, flux, the
    unlimited and limited new saturation and the limiter flags."""
    g, p = model.grid, model.prob
    A, f = reduced_system(model, s, mode)
    pN = solve_reduced(A, f)
    ph = reconstruct_pressure(model, pN)
    F = reconstruct_flux(g, p, ph, Mobility(g, p, s=s))
    s_new, flags = saturation_step(g, p, s, F, dt)
    return dict(A=A, f=f, pN=pN, ph=ph, F=F, s=s_new, flags=flags)
