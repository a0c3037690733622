"""Grid, P1 cell basis, quadrature and mobilities (oracle; test infrastructure).

Discrete space (Sec. 3.1): broken P^1 on a Cartesian grid.  On cell e with
centre b_e and sizes h_a the local coordinate is xi_a = 2 (x_a - b_a) / h_a in
[-1, 1]; the cell basis is L2-orthonormal:
    phi_0 = |e|^{-1/2},   phi_{a+1} = sqrt(3) xi_a |e|^{-1/2}   (a < d).
A field is stored SoA: coefficient k of cell c at index k*ncell + c.

Quadrature for integrands that are non-polynomial in the state (mobility,
fractional flow): tensor 2-point Gauss on cells (2^d points) and faces
(2^(d-1) points); exact for the quadratic mobility of P1 states.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

GP = 1.0 / math.sqrt(3.0)
SQ3 = math.sqrt(3.0)


class Grid:
    """Cartesian fine grid T_h with faces enumerated per axis (lo/hi cells)."""

    def __init__(self, prob):
        self.dim = d = prob.dim
        self.n = tuple(int(v) for v in prob.n)
        self.L = tuple(float(v) for v in prob.L)
        self.h = np.array([self.L[a] / self.n[a] for a in range(3)])
        self.vol = float(np.prod(self.h[:d]))
        self.ncell = int(np.prod(self.n))
        self.r = d + 1
        nx, ny, nz = self.n
        kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        self.ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
        self.centers = (self.ijk + 0.5) * self.h[None, :]
        self.faces = []
        off = 0
        for a in range(d):
            ext = list(self.n)
            ext[a] += 1
            k, j, i = np.meshgrid(np.arange(ext[2]), np.arange(ext[1]), np.arange(ext[0]),
                                  indexing="ij")
            idx = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1)
            ia = idx[:, a]
            lo_idx = idx.copy()
            lo_idx[:, a] -= 1
            lo = np.where(ia >= 1, self.cell_id(lo_idx), -1)
            hi = np.where(ia <= self.n[a] - 1, self.cell_id(np.minimum(idx, np.array(self.n) - 1)), -1)
            tang = [t for t in range(d) if t != a]
            area = float(np.prod([self.h[t] for t in tang])) if tang else 1.0
            hf = float(math.sqrt(sum(self.h[t] ** 2 for t in tang))) if tang else 1.0
            self.faces.append(dict(axis=a, lo=lo, hi=hi, gid=off + np.arange(len(lo)),
                                   area=area, hf=hf, tang=tang, idx=idx))
            off += len(lo)
        self.nface = off
        self.he = float(math.sqrt(sum(self.h[a] ** 2 for a in range(d))))   # diam(e)

    def cell_id(self, idx):
        nx, ny, _ = self.n
        return idx[:, 0] + nx * (idx[:, 1] + ny * idx[:, 2])

    # --- basis -----------------------------------------------------------
    def basis_at(self, xi):
        """Values of phi_0..phi_d at local points xi (npts, d); shape (npts, r)."""
        xi = np.atleast_2d(xi)
        out = np.empty((xi.shape[0], self.r))
        out[:, 0] = 1.0
        out[:, 1:] = SQ3 * xi[:, :self.dim]
        return out / math.sqrt(self.vol)

    def grad_basis(self):
        """Constant gradients of the basis, shape (r, d)."""
        g = np.zeros((self.r, self.dim))
        for a in range(self.dim):
            g[a + 1, a] = SQ3 * 2.0 / self.h[a] / math.sqrt(self.vol)
        return g

    def cell_qpts(self):
        """2-point Gauss tensor rule on the reference cell: points, weights."""
        pts = np.array(list(itertools.product([-GP, GP], repeat=self.dim)))
        w = np.full(len(pts), self.vol / len(pts))
        return pts, w

    def face_qpts(self, a, xi_a):
        """Gauss points on the face of a cell at xi_a = +-1 (local coords),
        and weights (sum = face area)."""
        f = self.faces[a]
        tang = f["tang"]
        tp = list(itertools.product([-GP, GP], repeat=len(tang)))
        pts = np.zeros((len(tp), self.dim))
        for q, t in enumerate(tp):
            pts[q, a] = xi_a
            for m, ax in enumerate(tang):
                pts[q, ax] = t[m]
        w = np.full(len(pts), f["area"] / len(pts))
        return pts, w

    def eval_field(self, u, c, xi):
        """Values of P1 field u (SoA) on cells c (array) at local points xi.
        Returns (len(c), npts)."""
        B = self.basis_at(xi)                       # (npts, r)
        coef = np.stack([u[k * self.ncell + c] for k in range(self.r)], axis=1)
        return coef @ B.T

    def vertices(self):
        return np.array(list(itertools.product([-1.0, 1.0], repeat=self.dim)))


# --- mobilities (eq. brooksCorey, eq. frationalFlow) ---------------------
def relperms(s, prob):
    """k_rw, k_ro at saturation s (clipped to [0, 1], where they are defined)."""
    sc = np.clip(s, 0.0, 1.0)
    if prob.relperm == 0:
        return sc, 1.0 - sc
    return sc ** prob.corey_w, (1.0 - sc) ** prob.corey_o


def mobilities(s, prob):
    """lambda_w = k_rw / eta_w, lambda_o = k_ro / eta_o, lambda = sum."""
    krw, kro = relperms(s, prob)
    lw = krw / prob.visc_w
    lo = kro / prob.visc_o
    return lw, lo, lw + lo


def total_mobility(s, prob):
    return mobilities(s, prob)[2]


def frac_flow(s, prob):
    lw, lo, lt = mobilities(s, prob)
    return lw / lt


def penalty_sigma(prob, k1, k2=None):
    """sigma_f = (c_f / max eta) * 2 a1 a2 / (a1 + a2), a_l = kappa on side l
    (eq. penaltyParam with the mobility-free constant of the Remark after it);
    on a one-sided (boundary) face sigma_f = (c_f / max eta) * a1."""
    c = prob.penalty_c / max(prob.visc_w, prob.visc_o)
    if k2 is None:
        return c * k1
    return c * 2.0 * k1 * k2 / (k1 + k2)


def mean_weights(prob, k1, k2):
    """Weights of the weighted mean {w} = w1 * om1 + w2 * om2.  SWIP (default):
    om1 = a2/(a1+a2), om2 = a1/(a1+a2); LITERAL: om_l = a_l/(a1+a2)."""
    if prob.weights == 0:
        return k2 / (k1 + k2), k1 / (k1 + k2)
    return k1 / (k1 + k2), k2 / (k1 + k2)
