"""Brute-force SWIP assembler for tiny grids (oracle; test infrastructure).

An independent, deliberately naive evaluation of b_h(v, w; lambda(s)) and
l_h(w) (Sec. 3.2, with the readings listed in ``pressure``): explicit loops
over cells, over neighbour pairs and over boundary faces, physical
coordinates, 4-point Gauss-Legendre tensor rules and point-wise basis
evaluation.  It shares only the relative-permeability law with the rest of
the oracle.  Used to pin the vectorized assembler on 2x2, 3x2 and 2x2x2 grids.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .fem import mobilities

_GX, _GW = np.polynomial.legendre.leggauss(4)


def _rule(lo, hi, axes_free, fixed):
    """Tensor Gauss points over the box [lo, hi] in axes_free; other coords fixed."""
    pts, wts = [], []
    for combo in itertools.product(range(4), repeat=len(axes_free)):
        x = np.array(fixed, dtype=float)
        wt = 1.0
        for m, ax in enumerate(axes_free):
            half = 0.5 * (hi[ax] - lo[ax])
            x[ax] = 0.5 * (hi[ax] + lo[ax]) + half * _GX[combo[m]]
            wt *= half * _GW[combo[m]]
        pts.append(x)
        wts.append(wt)
    return pts, wts


def brute_assemble(prob, s):
    d = prob.dim
    n = list(prob.n)
    h = [prob.L[a] / n[a] for a in range(3)]
    r = d + 1
    cells = list(itertools.product(*[range(n[a]) for a in range(d)]))
    nc = len(cells)

    def cid(idx):
        idx = list(idx) + [0] * (3 - len(idx))
        return idx[0] + n[0] * (idx[1] + n[1] * idx[2])

    vol = float(np.prod(h[:d]))

    def lo_hi(idx):
        lo = np.array([idx[a] * h[a] for a in range(d)])
        return lo, lo + np.array(h[:d])

    def phi(idx, k, x):
        lo, hi = lo_hi(idx)
        if k == 0:
            return 1.0 / math.sqrt(vol)
        a = k - 1
        xi = 2.0 * (x[a] - 0.5 * (lo[a] + hi[a])) / h[a]
        return math.sqrt(3.0) * xi / math.sqrt(vol)

    def gphi(idx, k):
        g = np.zeros(d)
        if k > 0:
            g[k - 1] = math.sqrt(3.0) * 2.0 / h[k - 1] / math.sqrt(vol)
        return g

    def sval(idx, x):
        c = cid(idx)
        return sum(s[k * nc + c] * phi(idx, k, x) for k in range(r))

    def lam(idx, x):
        return mobilities(np.array([sval(idx, x)]), prob)[2][0]

    kap = lambda idx: prob.perm[cid(idx)]
    cmax = prob.penalty_c / max(prob.visc_w, prob.visc_o)
    A = np.zeros((r * nc, r * nc))
    l = np.zeros(r * nc)
    dof = lambda idx, k: k * nc + cid(idx)

    for idx in cells:
        lo, hi = lo_hi(idx)
        pts, wts = _rule(lo, hi, list(range(d)), lo)
        for i in range(r):
            for j in range(r):
                gi, gj = gphi(idx, i), gphi(idx, j)
                A[dof(idx, i), dof(idx, j)] += sum(wt * lam(idx, x) * kap(idx) * (gi @ gj)
                                                   for x, wt in zip(pts, wts))
            l[dof(idx, i)] += sum(wt * prob.q1[cid(idx)] * phi(idx, i, x) for x, wt in zip(pts, wts))

    def face_gid(a, fidx):
        ext = list(n)
        ext[a] += 1
        off = 0
        for b in range(a):
            e2 = list(n)
            e2[b] += 1
            off += e2[0] * e2[1] * e2[2]
        f3 = list(fidx) + [0] * (3 - len(fidx))
        return off + f3[0] + ext[0] * (f3[1] + ext[1] * f3[2])

    for a in range(d):
        tang = [t for t in range(d) if t != a]
        hf = math.sqrt(sum(h[t] ** 2 for t in tang))
        nvec = np.zeros(d)
        nvec[a] = 1.0
        for idx in cells:
            lo, hi = lo_hi(idx)
            # interior face between idx (side 1) and its +a neighbour (side 2)
            if idx[a] + 1 < n[a]:
                nb = list(idx)
                nb[a] += 1
                nb = tuple(nb)
                fixed = lo.copy()
                fixed[a] = hi[a]
                pts, wts = _rule(lo, hi, tang, fixed)
                a1, a2 = kap(idx), kap(nb)
                if prob.weights == 0:
                    w1, w2 = a2 / (a1 + a2), a1 / (a1 + a2)
                else:
                    w1, w2 = a1 / (a1 + a2), a2 / (a1 + a2)
                sig = cmax * 2 * a1 * a2 / (a1 + a2)
                sides = [(idx, 1.0, w1, a1), (nb, -1.0, w2, a2)]
                for (ci, si, _, _) in sides:
                    for i in range(r):
                        for (cj, sj, _, _) in sides:
                            for j in range(r):
                                val = 0.0
                                for x, wt in zip(pts, wts):
                                    jv = si * phi(ci, i, x)
                                    jw = sj * phi(cj, j, x)
                                    mean_v = sum(wl * al * lam(cl, x) * (gphi(cl, i) @ nvec) * (cl == ci)
                                                 for (cl, _, wl, al) in sides)
                                    mean_w = sum(wl * al * lam(cl, x) * (gphi(cl, j) @ nvec) * (cl == cj)
                                                 for (cl, _, wl, al) in sides)
                                    val += wt * (sig / hf * jv * jw - mean_v * jw - mean_w * jv)
                                A[dof(ci, i), dof(cj, j)] += val
            # boundary faces of idx along a
            for side in (0, 1):
                if (side == 0 and idx[a] != 0) or (side == 1 and idx[a] != n[a] - 1):
                    continue
                fidx = list(idx)
                if side == 1:
                    fidx[a] += 1
                g = face_gid(a, fidx)
                nout = nvec * (1.0 if side == 1 else -1.0)
                fixed = lo.copy()
                fixed[a] = hi[a] if side == 1 else lo[a]
                pts, wts = _rule(lo, hi, tang, fixed)
                bt = prob.bc_type[g]
                val = prob.bc_val[g]
                if bt == 1:
                    for i in range(r):
                        l[dof(idx, i)] -= sum(wt * val * phi(idx, i, x) for x, wt in zip(pts, wts))
                elif bt == 2:
                    sig = cmax * kap(idx)
                    for i in range(r):
                        for j in range(r):
                            v = 0.0
                            for x, wt in zip(pts, wts):
                                v += wt * (sig / hf * phi(idx, i, x) * phi(idx, j, x)
                                           - lam(idx, x) * kap(idx) * (gphi(idx, i) @ nout) * phi(idx, j, x)
                                           - lam(idx, x) * kap(idx) * (gphi(idx, j) @ nout) * phi(idx, i, x))
                            A[dof(idx, i), dof(idx, j)] += v
                        l[dof(idx, i)] += sum(wt * (sig / hf * phi(idx, i, x)
                                                    - lam(idx, x) * kap(idx) * (gphi(idx, i) @ nout)) * val
                                              for x, wt in zip(pts, wts))
    return A, l
